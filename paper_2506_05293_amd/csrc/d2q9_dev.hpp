// D2Q9 node arithmetic for gfx950, in offset form.
//
// Populations are stored as offsets g_i = f_i - w_i (FP64, FP32 or FP16
// storage; FP32 arithmetic for the last two).  Every formula below is written
// on offsets so that no large constant is ever added to a small one:
//   rho = 1 + sum_i g_i,  j = sum_i c_i g_i  (sum_i w_i c_i = 0),
//   g_i^eq = w_i (drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u))      (Eq. 3)
// Numbering q: 0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1) 6 (-1,1)
// 7 (-1,-1) 8 (1,-1).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbm {

__host__ __device__ constexpr int cx(int q) {
  return q == 1 || q == 5 || q == 8 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy(int q) {
  return q == 2 || q == 5 || q == 6 ? 1 : (q == 4 || q == 7 || q == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp(int q) {
  return q == 0 ? 0 : (q <= 4 ? ((q + 1) & 3) + 1 : ((q - 3) & 3) + 5);
}
template <typename T>
__host__ __device__ constexpr T wgt(int q) {
  return q == 0 ? T(4) / T(9) : (q <= 4 ? T(1) / T(9) : T(1) / T(36));
}

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp");

// Per-node link word (uint32) built on the host from the geometry mask.
enum : uint32_t {
  LINK_BB_SHIFT = 0,      // bit q: population q is pulled by bounce-back
  LINK_FORCE_SHIFT = 9,   // bit 9+q: ... and its source is a body node
  LINK_SOLID = 1u << 24,  // the node itself is solid: not updated
  LINK_INLET = 1u << 25,  // Zou & He velocity column x = 0
  LINK_OUTLET = 1u << 26  // outflow column x = nx-1
};

// ---- storage conversion -----------------------------------------------------
// ld: plain load; ld_nt: load with the non-temporal hint; st: store with the
// non-temporal hint (each population is written once per step); st_cached:
// plain store (set-up kernels); stored: the value a store and a reload give
// (a kernel that keeps a state in registers between steps rounds it so).
template <typename S> struct Store;
template <> struct Store<double> {
  using T = double;
  __device__ static T ld(const double* p) { return *p; }
  __device__ static T ld_nt(const double* p) { return __builtin_nontemporal_load(p); }
  __device__ static void st(double* p, T v) { __builtin_nontemporal_store(v, p); }
  __device__ static void st_cached(double* p, T v) { *p = v; }
  __device__ static T stored(T v) { return v; }
};
template <> struct Store<float> {
  using T = float;
  __device__ static T ld(const float* p) { return *p; }
  __device__ static T ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
  __device__ static void st(float* p, T v) { __builtin_nontemporal_store(v, p); }
  __device__ static void st_cached(float* p, T v) { *p = v; }
  __device__ static T stored(T v) { return v; }
};
// FP16 storage rounds the FP32 value the arithmetic left (round to nearest
// even): to_half keeps the compiler from fusing the multiply-add that made v
// with the conversion (a mixed-precision FMA rounds once, straight to FP16,
// and would make one kernel's stored value differ from another's).
__device__ __forceinline__ __half to_half(float v) {
  asm volatile("" : "+v"(v));
  return __float2half_rn(v);
}
template <> struct Store<__half> {
  using T = float;
  __device__ static T ld(const __half* p) { return __half2float(*p); }
  __device__ static T ld_nt(const __half* p) {
    return __half2float(__ushort_as_half(
        __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p))));
  }
  __device__ static void st(__half* p, T v) {
    __builtin_nontemporal_store(__half_as_ushort(to_half(v)), reinterpret_cast<unsigned short*>(p));
  }
  __device__ static void st_cached(__half* p, T v) { *p = to_half(v); }
  __device__ static T stored(T v) { return __half2float(to_half(v)); }
};

// ---- arithmetic shared by every kernel ------------------------------------------
// The node arithmetic below is written with explicit fused multiply-adds and
// with contraction switched off, so the compiler cannot fuse a product and a
// sum differently in different kernels: every kernel that runs these
// functions (one step per launch, two steps per launch, the batch, the
// outlet blocks) computes the same IEEE operations on the same values.
template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
  if constexpr (sizeof(T) == 8)
    return __builtin_fma(a, b, c);
  else
    return __builtin_fmaf(a, b, c);
}

// 1 / rho: the hardware reciprocal in FP32 (within 1 ulp), a division in FP64.
template <typename T>
__device__ __forceinline__ T inv_rho(T rho) {
  if constexpr (sizeof(T) == 8)
    return T(1) / rho;
  else
    return __builtin_amdgcn_rcpf(rho);
}

// ---- moments -----------------------------------------------------------------
template <typename T>
struct Macro {
  T drho, rho, jx, jy;
};

template <typename T>
__device__ __forceinline__ Macro<T> macro(const T g[9]) {
#pragma clang fp contract(off)
  Macro<T> m;
  m.drho = ((g[0] + g[2] + g[4]) + (g[1] + g[3])) + ((g[5] + g[7]) + (g[6] + g[8]));
  m.rho = T(1) + m.drho;
  m.jx = (g[1] - g[3]) + ((g[5] - g[7]) + (g[8] - g[6]));
  m.jy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
  return m;
}

// ---- BGK (Eq. 2) in offset form -------------------------------------------------
// g_eq = w (drho + rho (c.u (3 + 9/2 c.u) - 3/2 u.u)); c.u is a signed sum of
// u_x and u_y (no products by 0 or 1).
template <typename T>
__device__ __forceinline__ void collide_bgk(T g[9], T omega) {
#pragma clang fp contract(off)
  const Macro<T> m = macro(g);
  const T inv = inv_rho(m.rho);
  const T ux = m.jx * inv, uy = m.jy * inv;
  const T usq = T(1.5) * fmadd(ux, ux, uy * uy);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const T cu = cx(q) == 0 ? (cy(q) == 0 ? T(0) : (cy(q) > 0 ? uy : -uy))
                            : (cy(q) == 0 ? (cx(q) > 0 ? ux : -ux)
                                          : (cx(q) > 0 ? ux : -ux) + (cy(q) > 0 ? uy : -uy));
    const T poly = q == 0 ? -usq : fmadd(cu, fmadd(T(4.5), cu, T(3)), -usq);
    const T geq = wgt<T>(q) * fmadd(m.rho, poly, m.drho);
    g[q] = fmadd(-omega, g[q] - geq, g[q]);
  }
}

// ---- MRT in offset form ---------------------------------------------------------
// Orthogonal basis rho, e, eps, jx, qx, jy, qy, pxx, pxy with squared norms
// 9, 36, 36, 6, 12, 6, 12, 4, 4.  Offsets shift e by -2 and eps by +1 (the
// moments of the weights), so the equilibria below are offsets as well:
//   e^eq = -2 drho + 3 |j|^2/rho,  eps^eq = drho - 3 |j|^2/rho,
//   qx^eq = -jx, qy^eq = -jy, pxx^eq = (jx^2 - jy^2)/rho, pxy^eq = jx jy/rho.
// Only the six non-conserved moments relax; the change is mapped back by
// M^T diag(1/norm^2).
template <typename T>
struct MrtRates {
  T s_e, s_eps, s_q, s_nu;
};

template <typename T>
__device__ __forceinline__ void collide_mrt(T g[9], const MrtRates<T>& r) {
#pragma clang fp contract(off)
  const Macro<T> m = macro(g);
  const T inv = inv_rho(m.rho);
  const T jy2 = m.jy * m.jy;
  const T j2 = fmadd(m.jx, m.jx, jy2) * inv;
  const T sa = (g[1] + g[2]) + (g[3] + g[4]);
  const T sd = (g[5] + g[6]) + (g[7] + g[8]);
  const T e = fmadd(T(2), sd, fmadd(T(-4), g[0], -sa));
  const T eps = fmadd(T(4), g[0], fmadd(T(-2), sa, sd));
  const T d57 = g[5] - g[7], d86 = g[8] - g[6], d68 = g[6] - g[8];
  const T qx = fmadd(T(2), g[3] - g[1], d57 + d86);
  const T qy = fmadd(T(2), g[4] - g[2], d57 + d68);
  const T pxx = (g[1] + g[3]) - (g[2] + g[4]);
  const T pxy = (g[5] + g[7]) - (g[6] + g[8]);
  const T de = r.s_e * (e - fmadd(T(-2), m.drho, T(3) * j2)) * T(1.0 / 36.0);
  const T dp = r.s_eps * (eps - fmadd(T(-3), j2, m.drho)) * T(1.0 / 36.0);
  const T dqx = r.s_q * (qx + m.jx) * T(1.0 / 12.0);
  const T dqy = r.s_q * (qy + m.jy) * T(1.0 / 12.0);
  const T dxx = r.s_nu * fmadd(-fmadd(m.jx, m.jx, -jy2), inv, pxx) * T(0.25);
  const T dxy = r.s_nu * fmadd(-(m.jx * m.jy), inv, pxy) * T(0.25);
  const T a = fmadd(T(-2), dp, -de);    // shared by q = 1..4
  const T b = fmadd(T(2), de, dp);      // shared by q = 5..8
  g[0] = fmadd(T(-4), dp - de, g[0]);
  g[1] -= fmadd(T(-2), dqx, a) + dxx;
  g[2] -= fmadd(T(-2), dqy, a) - dxx;
  g[3] -= fmadd(T(2), dqx, a) + dxx;
  g[4] -= fmadd(T(2), dqy, a) - dxx;
  g[5] -= ((b + dqx) + dqy) + dxy;
  g[6] -= ((b - dqx) + dqy) - dxy;
  g[7] -= ((b - dqx) - dqy) + dxy;
  g[8] -= ((b + dqx) - dqy) - dxy;
}

// ---- Zou & He columns (Sec. 2.2), offsets ----------------------------------------
// Velocity inlet at x = 0, prescribed (u, 0), unknowns 1, 5, 8.  The weight
// part of rho_0 + 2 rho_- is exactly 1, so
//   rho = (1 + drho_0 + 2 drho_-) / (1 - u),
//   g1 = g3 + (2/3) rho u,  g5 = g7 + (g4 - g2)/2 + rho u/6,
//   g8 = g6 - (g4 - g2)/2 + rho u/6.
template <typename T>
__device__ __forceinline__ void zouhe_inlet(T g[9], T u) {
#pragma clang fp contract(off)
  const T d0 = g[0] + g[2] + g[4];
  const T dm = g[3] + g[6] + g[7];
  const T drho = (fmadd(T(2), dm, d0) + u) / (T(1) - u);
  const T ru = (T(1) + drho) * u;
  const T h = T(0.5) * (g[4] - g[2]);
  g[1] = fmadd(ru, T(2.0 / 3.0), g[3]);
  g[5] = fmadd(ru, T(1.0 / 6.0), g[7] + h);
  g[8] = fmadd(ru, T(1.0 / 6.0), g[6] - h);
}

// Pressure outlet at x = nx-1, prescribed rho_out and v = 0, unknowns 3, 6, 7:
//   rho u = rho_0 + 2 rho_+ - rho_out = drho_0 + 2 drho_+ + (1 - rho_out),
//   g3 = g1 - (2/3) rho u,  g6 = g8 + (g4 - g2)/2 - rho u/6,
//   g7 = g5 - (g4 - g2)/2 - rho u/6.
template <typename T>
__device__ __forceinline__ void zouhe_outlet(T g[9], T one_minus_rho_out) {
#pragma clang fp contract(off)
  const T d0 = g[0] + g[2] + g[4];
  const T dp = g[1] + g[5] + g[8];
  const T ru = fmadd(T(2), dp, d0) + one_minus_rho_out;
  const T h = T(0.5) * (g[4] - g[2]);
  g[3] = fmadd(ru, T(-2.0 / 3.0), g[1]);
  g[6] = fmadd(ru, T(-1.0 / 6.0), g[8] + h);
  g[7] = fmadd(ru, T(-1.0 / 6.0), g[5] - h);
}

// Right boundary with a prescribed state (rho, u, v), offset form (drho =
// rho - 1): f_0 is corrected so that the node carries the density exactly
// (Eq. 29, g_0 = f_0 + rho (1 + u) - (rho_0 + 2 rho_+)), the unknowns 3, 6, 7
// follow from Eqs. 8-10 with the transverse velocity.
template <typename T>
__device__ __forceinline__ void outlet_state(T g[9], T drho, T u, T v) {
#pragma clang fp contract(off)
  const T d0 = g[0] + g[2] + g[4];
  const T dp = g[1] + g[5] + g[8];
  g[0] += fmadd(drho, u, drho + u) - fmadd(T(2), dp, d0);
  const T rho = T(1) + drho;
  const T ru = rho * u, rv = rho * v;
  const T h = T(0.5) * (g[4] - g[2]);
  g[3] = fmadd(ru, T(-2.0 / 3.0), g[1]);
  g[6] = fmadd(T(0.5), rv, fmadd(ru, T(-1.0 / 6.0), g[8] + h));
  g[7] = fmadd(T(-0.5), rv, fmadd(ru, T(-1.0 / 6.0), g[5] - h));
}

// ---- SplitMix64, counter form ------------------------------------------------------
// Output k (k >= 1) of the stream seeded with s is the finaliser applied to
// s + k * 0x9e3779b97f4a7c15 (Steele, Lea & Flood 2014).
__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline double unit_double(uint64_t r) {
  return double(r >> 11) * (1.0 / 9007199254740992.0);  // 2^-53
}

}  // namespace lbm
