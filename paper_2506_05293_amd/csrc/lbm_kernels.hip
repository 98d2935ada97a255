// HIP kernels of the D2Q9 time step for gfx950.
//
// Three kernels take the step: k_step3 advances three steps per launch
// (Zou & He or neural outflow, FP32 and FP16 offsets; the default), k_step2
// two (every outflow and precision), k_step one (described first below).
// All run the same node code, so the populations agree bit for bit.
//
// One launch of k_step advances the lattice by one step (Sec. 2.1 Eq. 1 in pull form):
// every fluid node gathers the post-collision populations of its neighbours
// from buffer A (half-way bounce-back where the source is a wall or a solid,
// Eq. 12), completes the inlet / outlet column (Sec. 2.2; Sec. 3.1 Eq. 16;
// Sec. 4, Eqs. 18-29),
// collides (Eq. 2 or MRT) and writes its post-collision populations to B.
// The same launch produces the momentum-exchange force of the step
// (Eqs. 14-15) and the mass, as per-workgroup partial sums.
//
// Grid layout (block ids; the bulk tiles are remapped per XCD, see xcd_remap):
//   0                     level-2 reduction (FP64, fixed order) of the step
//                         before the previous one into the accumulators;
//   1 .. kReducers        level-1 reduction of the previous step's slots;
//   next n_nn             outlet blocks (neural or characteristic outflow),
//                         64 outlet rows each;
//   up to nspecial        padding to a multiple of 8 (empty slots);
//   the rest              bulk tiles, x fastest.
//
// Memory layout: population q of node (x, y) at q*plane + y*pitch + x, with
// pitch a multiple of 256 elements; offsets f - w stored in S (f for FP64).
#include <type_traits>

#include "d2q9_dev.hpp"
#include "lbm_internal.hpp"
#include "mlp_dev.hpp"
#include "node_dev.hpp"

namespace lbm {

// Workgroups are dispatched to the eight XCDs round-robin by blockIdx; give
// each XCD contiguous runs of tiles so that the cache lines two x-adjacent
// tiles share (the pull reads one element past each tile edge) meet in the
// same L2.  Either one band of n/8 tiles per XCD, or chunks of S tiles dealt
// to the XCDs in turn (XCD x takes chunks x, x + 8, ...; the tail after the
// last full round in bands).  Which one is the host's choice (xcd_chunk).
#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 1
#endif
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  if constexpr (!LBM_XCD_REMAP) return bid;
  const int q = n >> 3, r = n & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}
__device__ __forceinline__ int xcd_remap_chunks(int bid, int n, int S) {
  const int full = n / (8 * S) * (8 * S);
  if (bid >= full) return full + xcd_remap(bid - full, n - full);
  const int x = bid & 7, k = bid >> 3;
  return ((k / S) * 8 + x) * S + k % S;
}

// Optional occupancy request for the step kernel (waves per SIMD).
#ifdef LBM_WAVES_PER_EU
#define LBM_STEP_ATTR __attribute__((amdgpu_waves_per_eu(LBM_WAVES_PER_EU, LBM_WAVES_PER_EU)))
#else
#define LBM_STEP_ATTR
#endif

// Partial sums are kept per wave: lane 0 of wave w of workgroup v writes
// slot 4 v + w (no barrier, so waves retire independently).
template <typename T>
__device__ __forceinline__ void wave_partials(T a, T b, T c, T d, T* block_slots) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  d = wave_sum(d);
  if ((threadIdx.x & 63) == 0) {
    T* out = block_slots + kPartials * (threadIdx.x >> 6);
    out[0] = a;
    out[1] = b;
    out[2] = c;
    out[3] = d;
  }
}

// Block sum of four FP64 values in a fixed order; thread 0 gets the result.
__device__ __forceinline__ void block_sum4(double s[4], double out[4]) {
  __shared__ double red[kWaves][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = wave_sum(s[k]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) red[threadIdx.x >> 6][k] = s[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// FP64 sum of slots [b0, b1) of one step's partials: thread t adds slots
// b0 + t, b0 + t + 256, ... in that order (one vector load per slot), then
// the workgroup combines the threads in a fixed order, so the result does
// not depend on timing.
template <typename T>
__device__ void sum_slots(const T* __restrict__ part, int b0, int b1, double out[4]) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  const v4* slot = reinterpret_cast<const v4*>(part);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int b = b0 + int(threadIdx.x); b < b1; b += kBlock) {
    const v4 p = slot[b];
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] += double(p[k]);
  }
  block_sum4(s, out);
}

// Fold one step's total (fx, fy, sum of rho - 1, fallbacks) into the
// accumulators and the force history (thread 0 only).
__device__ void commit_step(const double t[4], const StepLaunch& L) {
  Acc* acc = L.acc;
  acc->fx = t[0];
  acc->fy = t[1];
  acc->fx_sum += t[0];
  acc->fy_sum += t[1];
  acc->mass = L.n_fluid + t[2];
  acc->fallback += t[3];
  if (!isfinite(t[0]) || !isfinite(t[1]) || !isfinite(t[2])) acc->nonfinite = 1;
  const int64_t n = acc->n_reduced;
  if (n < L.hist_cap) {
    L.hist[3 * n + 0] = t[0];
    L.hist[3 * n + 1] = t[1];
    L.hist[3 * n + 2] = L.n_fluid + t[2];
  }
  acc->n_reduced = n + 1;
}

// Level 2: the kReducers sums of one step -> accumulators.
__device__ void reduce_level2(const double* __restrict__ lvl, const StepLaunch& L) {
  double s[4] = {0.0, 0.0, 0.0, 0.0}, t[4];
  if (threadIdx.x < kReducers) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = lvl[threadIdx.x * 4 + k];
  }
  block_sum4(s, t);
  if (threadIdx.x == 0) commit_step(t, L);
}

// Level 1: reducer r sums its slice of the previous step's slots.
template <typename T>
__device__ void reduce_level1(const T* __restrict__ part, int r, const StepLaunch& L) {
  const int per = (L.nslots + kReducers - 1) / kReducers;
  const int b0 = min(r * per, L.nslots), b1 = min(b0 + per, L.nslots);
  double t[4];
  sum_slots(part, b0, b1, t);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) L.lvl_w[r * 4 + k] = t[k];
  }
}

template <typename S, int MRT, int PATH>
__device__ __forceinline__ void bulk_block(const StepLaunch& L, int tile,
                                           typename Store<S>::T* part) {
  using T = typename Store<S>::T;
  const int tx = tile % L.ntx, ty = tile / L.ntx;
  T fx = T(0), fy = T(0), dm = T(0);
  if constexpr (PATH == PATH_SCALAR) {
    const int x = tx * kChunk + threadIdx.x;
    if (x < L.nx) bulk_node<S, MRT>(L, tx, x, ty, fx, fy, dm);
  } else {
    const int lane = threadIdx.x & 63;
    const int y = ty * tile_rows(PATH) + (threadIdx.x >> 6);
    if (y < L.ny) bulk_row<S, MRT>(L, tx, y, lane, fx, fy, dm);   // wave-uniform
  }
  wave_partials(fx, fy, dm, T(0), part);
}

// ---- neural outlet block ----------------------------------------------------------
constexpr int kStRows = kNnRows + 2;   // staged rows y0-1 .. y0+64
constexpr int kStCols = 5;             // staged columns nx-5 .. nx-1

template <typename T>
struct alignas(16) NnSmem {
  union {
    T st[9 * kStRows * kStCols];       // A around the outlet, rows y0-1..y0+64
    MlpH H;                            // network activations (after staging)
  } u;
  MlpX X;
  T prev[kNnRows * 4];                 // g3, g6, g7 and drho at x = L-1
};

// Eq. 16 at the outlet node: g holds its pulled populations (the unknowns
// 3, 6, 7 are replaced), o the network's standardised outputs, prev the
// pre-collision g3, g6, g7 and density offset of column L-1.  The node keeps
// g_i = f_i(L-1) + s_i, s = o sd_out + mu_out, if every reconstructed
// population is positive and the density moves by less than mass_bound
// (FP32 tests); otherwise Zou & He.  Returns true if the reconstruction is
// kept.
template <typename T>
__device__ __forceinline__ bool nn_reconstruct(const MlpDev* __restrict__ w, const float* o,
                                               const T* prev, T g[9], T one_minus_rho_out) {
#pragma clang fp contract(off)
  T r[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) r[q] = g[q];
  r[3] = prev[0] + T(fmaf(o[0], w->sd_out[0], w->mu_out[0]));
  r[6] = prev[1] + T(fmaf(o[1], w->sd_out[1], w->mu_out[1]));
  r[7] = prev[2] + T(fmaf(o[2], w->sd_out[2], w->mu_out[2]));
  const float drg = float(macro(r).drho);
  const bool ok = float(r[3] + wgt<T>(3)) > 0.f && float(r[6] + wgt<T>(6)) > 0.f &&
                  float(r[7] + wgt<T>(7)) > 0.f && fabsf(drg - float(prev[3])) < w->mass_bound;
  if (ok) {
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = r[q];
  } else {
    zouhe_outlet(g, one_minus_rho_out);
  }
  return ok;
}

template <typename S, int MRT>
__device__ void nn_block(const StepLaunch& L, int nb, NnSmem<typename Store<S>::T>& sm,
                         typename Store<S>::T* part) {
  using T = typename Store<S>::T;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const MlpDev* __restrict__ w = L.mlp;
  const int y0 = nb * kNnRows;
  const int xs0 = L.nx - kStCols;

  // 1. stage A[q][y0-1 .. y0+64][nx-5 .. nx-1] in LDS
  for (int i = threadIdx.x; i < 9 * kStRows * kStCols; i += kBlock) {
    const int q = i / (kStRows * kStCols);
    const int rem = i - q * (kStRows * kStCols);
    const int r = rem / kStCols;
    const int c = rem - r * kStCols;
    int y = y0 - 1 + r;
    if (L.yper)
      y = (y + L.ny) % L.ny;
    else
      y = min(max(y, 0), L.ny - 1);    // such rows are only reached by bounce-back
    sm.u.st[i] = Store<S>::ld(A + int64_t(q) * L.plane + int64_t(y) * L.pitch + xs0 + c);
  }
  __syncthreads();

  // 2. pull the pre-collision populations of columns L-3 .. L (k = 0 .. 3)
  const int j = threadIdx.x & 63;
  const int k = threadIdx.x >> 6;
  const int y = y0 + j;
  const int x = L.nx - 4 + k;
  const bool active = y < L.ny;
  const uint32_t lk = active ? L.links[int64_t(y) * L.pitch + x] : LINK_SOLID;
  T g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const bool bb = (lk >> q) & 1u;
    const int c = bb ? k + 1 : min(k + 1 - cx(q), kStCols - 1);   // outlet unknowns: any
    const int r = bb ? j + 1 : j + 1 - cy(q);
    const int qq = bb ? opp(q) : q;
    g[q] = sm.u.st[(qq * kStRows + r) * kStCols + c];
  }
  T fx = T(0), fy = T(0), dm = T(0), nfb = T(0);
  if (k < 3) {
    // features of column x = L-1-jc, feature index 9 jc + q
    const int jc = 2 - k;
    const bool use = active && !(lk & LINK_SOLID);
#pragma unroll
    for (int q = 0; q < 9; ++q)
      sm.X.x[j * kXPitch + 9 * jc + q] = use ? feature_bf16(w, 9 * jc + q, float(g[q])) : 0;
    if (k == 0) {
#pragma unroll
      for (int f = 27; f < 32; ++f) sm.X.x[j * kXPitch + f] = 0;
    }
    if (k == 2) {
      sm.prev[j * 4 + 0] = g[3];
      sm.prev[j * 4 + 1] = g[6];
      sm.prev[j * 4 + 2] = g[7];
      sm.prev[j * 4 + 3] = macro(g).drho;
    }
  }
  __syncthreads();

  // 3. the network on the 64 rows (MFMA)
  mlp_tile(w, sm.X, sm.u.H);

  // 4. reconstruct the outlet node, fall back to Zou & He, collide, store
  if (k == 3 && active && !(lk & LINK_SOLID)) {
    add_force(lk, g, fx, fy);
    if (!nn_reconstruct(w, &sm.u.H.o[j * 4], &sm.prev[j * 4], g, T(L.one_minus_rho_out)))
      nfb = T(1);
    dm = macro(g).drho;
    collide<T, MRT>(g, L);
    const int64_t row = int64_t(y) * L.pitch + x;
#pragma unroll
    for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row, g[q]);
  }
  wave_partials(fx, fy, dm, nfb, part);
}


// ---- characteristic outlet block (Sec. 4, Eqs. 18-29) ------------------------
// 64 outlet rows per workgroup.  The state of the time level is the moments of
// the stored post-collision populations (collision conserves them); columns
// nx-3 .. nx-1 of rows y0-2 .. y0+65 are staged and reduced to (drho, u, v),
// then one thread per row takes the gradients (second-order one-sided in x,
// central in y), the tuning network if any, the LODI
// time derivatives with L_1 of Eq. 27, a forward Euler step, and rebuilds the
// unknown populations for that state before collision.  Lateral boundaries
// are periodic (the library rejects walls for this outflow).
constexpr int kCbRows = kNnRows + 4;
constexpr int kCbCols = 3;
constexpr int kCbUnits = kCbcHidden / kWaves;   // hidden units per wave and row

// LDS of the tuning network evaluated for 64 rows.
template <typename T>
struct alignas(16) CbcNetSmem {
  T feat[kNnRows * kCbcIn];              // network inputs per row
  T h1[kNnRows * kCbcHidden];            // first hidden layer
  T ps[kNnRows * kWaves * 2];            // per-wave partial sums of s_0, s_1
};

template <typename T>
struct alignas(16) CbcSmem {
  T st[9 * kCbRows * kCbCols];           // A at columns nx-3 .. nx-1, rows y0-2 .. y0+65
  T mo[3 * kCbCols * kCbRows];           // [k][column][row]: drho, u, v
  CbcNetSmem<T> net;
};

template <typename T>
__device__ __forceinline__ T sigmoid_t(T s) {
  if constexpr (sizeof(T) == 8)
    return T(1) / (T(1) + exp(-s));
  else
    return T(1) / (T(1) + expf(-s));
}

// Moments (drho, u, v) of the nodes of three consecutive columns c0 .. c0+2
// of a staged tile src[q][R][C] into mo[k][3][R] (all R rows).
template <typename T, int R, int C>
__device__ __forceinline__ void tile_moments(const T* src, int c0, T* mo) {
#pragma clang fp contract(off)
  for (int i = threadIdx.x; i < R * 3; i += kBlock) {
    const int r = i / 3, cc = i - (i / 3) * 3;
    T g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = src[(q * R + r) * C + c0 + cc];
    const Macro<T> m = macro(g);
    mo[(0 * 3 + cc) * R + r] = m.drho;
    mo[(1 * 3 + cc) * R + r] = m.jx / m.rho;
    mo[(2 * 3 + cc) * R + r] = m.jy / m.rho;
  }
}

// Gradients (p_x, u_x, v_x, p_y, u_y, v_y) at the outlet node of row r of a
// moment tile mo[k][3][R] (columns L-2, L-1, L): second-order one-sided in x,
// central in y (periodic rows are staged wrapped).
template <typename T, int R>
__device__ __forceinline__ void cbc_gradients(const T* mo, int r, T g[6]) {
#pragma clang fp contract(off)
  const T cs2 = T(1.0 / 3.0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T* m = mo + k * 3 * R;
    const T gx = T(0.5) * (T(3) * m[2 * R + r] - T(4) * m[R + r] + m[r]);
    const T gy = T(0.5) * (m[2 * R + r + 1] - m[2 * R + r - 1]);
    g[k] = k == 0 ? cs2 * gx : gx;
    g[3 + k] = k == 0 ? cs2 * gy : gy;
  }
}

template <typename T>
__device__ __forceinline__ T leaky_t(T x, T a) {
  return x > T(0) ? x : a * x;
}

// The tuning network (Sec. 4.2) on 64 rows, spread over the workgroup:
// thread j < 64 has written the nine standardised features of row j into
// net.feat; each wave takes kCbUnits of the hidden units of every row and
// leaves partial output sums, added in a fixed order.  Every thread calls
// it (it holds barriers); thread j < 64 gets sigma and kappa_2 of row j.
template <typename T>
__device__ __forceinline__ void cbc_network(const CbcDev* __restrict__ c, CbcNetSmem<T>& net,
                                            T& sigma, T& kappa2) {
#pragma clang fp contract(off)
  __syncthreads();
  const int rr = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T a = T(c->leaky);
#pragma unroll 1
  for (int u = 0; u < kCbUnits; ++u) {
    const int o = w * kCbUnits + u;
    T s = T(c->b1[o]);
#pragma unroll
    for (int i = 0; i < kCbcIn; ++i) s += T(c->w1[o * kCbcIn + i]) * net.feat[rr * kCbcIn + i];
    net.h1[rr * kCbcHidden + o] = leaky_t(s, a);
  }
  __syncthreads();
  T p0 = T(0), p1 = T(0);
#pragma unroll 1
  for (int u = 0; u < kCbUnits; ++u) {
    const int o = w * kCbUnits + u;
    T s = T(c->b2[o]);
#pragma unroll 4
    for (int k = 0; k < kCbcHidden; ++k) s += T(c->w2[o * kCbcHidden + k]) * net.h1[rr * kCbcHidden + k];
    const T h = leaky_t(s, a);
    p0 += T(c->w3[o]) * h;
    p1 += T(c->w3[kCbcHidden + o]) * h;
  }
  net.ps[(rr * kWaves + w) * 2 + 0] = p0;
  net.ps[(rr * kWaves + w) * 2 + 1] = p1;
  __syncthreads();
  if (threadIdx.x < kNnRows) {
    const T* q = net.ps + threadIdx.x * kWaves * 2;
    const T s0 = T(c->b3[0]) + ((q[0] + q[2]) + (q[4] + q[6]));
    const T s1 = T(c->b3[1]) + ((q[1] + q[3]) + (q[5] + q[7]));
    sigma = T(c->sigma_scale) * sigmoid_t(s0) + T(c->sigma_shift);
    kappa2 = T(c->kappa_scale) * sigmoid_t(s1) + T(c->kappa_shift);
  }
}

// Network features of one row: the gradients and the previous step's time
// derivatives (p_t, u_t, v_t), standardised.
template <typename T>
__device__ __forceinline__ void cbc_features(const CbcDev* __restrict__ c, const T g[6],
                                             const T prev[3], T* feat) {
#pragma clang fp contract(off)
#pragma unroll
  for (int i = 0; i < kCbcIn; ++i) {
    const T f = i < 6 ? g[i] : prev[i - 6];
    feat[i] = (f - T(c->mu_in[i])) / T(c->sd_in[i]);
  }
}

// Eqs. 18-28 at one outlet row: from the gradients g, the state (drho, u, v)
// and sigma, kappa_2, the LODI time derivatives; returns the new state by
// forward Euler in st and (p_t, u_t, v_t) in dt.
template <typename T>
__device__ __forceinline__ void cbc_lodi(const CbcDev* __restrict__ c, const T g6[6], T drho, T u,
                                         T v, T sigma, T kappa2, T st[3], T dt[3]) {
#pragma clang fp contract(off)
  const T p_x = g6[0], u_x = g6[1], v_x = g6[2], p_y = g6[3], u_y = g6[4], v_y = g6[5];
  const T cs2 = T(1.0 / 3.0), cs = T(0.57735026918962576451);
  const T rho = T(1) + drho, p = cs2 * rho;
  // Eqs. 21-26 (readings: dp/dx in L_1, L_5; du/dy in T_1, T_5)
  const T L3 = u * v_x;
  const T L5 = (u + cs) * (p_x + rho * cs * u_x);
  const T T1 = -(v * p_y + p * v_y - rho * cs * v * u_y);
  const T T3 = -(v * v_y + p_y / rho);
  const T T5 = -(v * p_y + p * v_y + rho * cs * v * u_y);
  // Eqs. 27-28 with T_1,exact = 0
  const T L1 = sigma * T(c->kappa1_coef) * cs2 * (drho - T(c->rho_inf_m1)) - kappa2 * T1 + T1;
  // Eqs. 18-20
  const T rho_t = (-(L5 + L1) + (T5 + T1)) / (T(2) * cs2);
  const T u_t = (-(L5 - L1) + (T5 - T1)) / (T(2) * rho * cs);
  const T v_t = -L3 + T3;
  dt[0] = cs2 * rho_t;
  dt[1] = u_t;
  dt[2] = v_t;
  st[0] = drho + rho_t;
  st[1] = u + u_t;
  st[2] = v + v_t;
}

template <typename S, int MRT>
__device__ void cbc_block(const StepLaunch& L, int nb, CbcSmem<typename Store<S>::T>& sm,
                          typename Store<S>::T* part) {
  using T = typename Store<S>::T;
  constexpr int R = kCbRows, NC = kCbCols;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const CbcDev* __restrict__ c = L.cbc;
  const int y0 = nb * kNnRows;
  const int xs0 = L.nx - NC;

  // 1. stage A[q][y0-2 .. y0+65][nx-3 .. nx-1] (rows wrapped: periodic laterals)
  for (int i = threadIdx.x; i < 9 * R * NC; i += kBlock) {
    const int q = i / (R * NC);
    const int rem = i - q * (R * NC);
    const int r = rem / NC;
    const int cc = rem - r * NC;
    const int y = (y0 - 2 + r + 2 * L.ny) % L.ny;
    sm.st[i] = Store<S>::ld(A + int64_t(q) * L.plane + int64_t(y) * L.pitch + xs0 + cc);
  }
  __syncthreads();
  // 2. the state (drho, u, v) of the staged nodes
  tile_moments<T, R, NC>(sm.st, 0, sm.mo);
  __syncthreads();

  const int j = threadIdx.x;
  const int y = y0 + j;
  const bool row = j < kNnRows && y < L.ny;
  double* dts = L.cbc_dt + 4 * int64_t(row ? y : 0);
  T sigma = T(c->sigma), kappa2 = T(c->kappa2);
  // 3. the tuning network, spread over the workgroup (uniform branch)
  if (c->has_net) {
    if (j < kNnRows) {
      T g[6];
      cbc_gradients<T, R>(sm.mo, j + 2, g);
      const T prev[3] = {row ? T(dts[0]) : T(0), row ? T(dts[1]) : T(0), row ? T(dts[2]) : T(0)};
      cbc_features(c, g, prev, &sm.net.feat[j * kCbcIn]);
    }
    cbc_network(c, sm.net, sigma, kappa2);
  }

  // 4. one thread per row: LODI update, reconstruction, collision
  T fx = T(0), fy = T(0), dm = T(0);
  const int x = L.nx - 1;
  if (row) {
    const uint32_t lk = L.links[int64_t(y) * L.pitch + x];
    if (!(lk & LINK_SOLID)) {
      const int r = j + 2;
      T g6[6], nst[3], dt[3];
      cbc_gradients<T, R>(sm.mo, r, g6);
      cbc_lodi(c, g6, sm.mo[(0 * NC + 2) * R + r], sm.mo[(1 * NC + 2) * R + r],
               sm.mo[(2 * NC + 2) * R + r], sigma, kappa2, nst, dt);
      dts[0] = double(dt[0]);
      dts[1] = double(dt[1]);
      dts[2] = double(dt[2]);
      // post-streaming populations of the outlet node
      T g[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const bool bb = (lk >> q) & 1u;
        const int cc = bb ? 2 : min(2 - cx(q), 2);      // unknowns: replaced below
        const int rr = bb ? r : r - cy(q);
        g[q] = sm.st[((bb ? opp(q) : q) * R + rr) * NC + cc];
      }
      outlet_state(g, nst[0], nst[1], nst[2]);   // forward Euler, Eq. 29, Eqs. 8-10
      add_force(lk, g, fx, fy);
      dm = macro(g).drho;
      collide<T, MRT>(g, L);
      const int64_t row_off = int64_t(y) * L.pitch + x;
#pragma unroll
      for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row_off, g[q]);
    }
  }
  wave_partials(fx, fy, dm, T(0), part);
}

// ---- the step kernel --------------------------------------------------------------
// OUT selects the outlet: 0 Zou & He in the bulk node code, OUTLET_NN or
// OUTLET_CBC in dedicated outlet blocks; each variant carries only its own
// registers and LDS.
template <typename S, int MRT, int OUT, int PATH>
__global__ void __launch_bounds__(kBlock) LBM_STEP_ATTR k_step(const StepLaunch L) {
  using T = typename Store<S>::T;
  constexpr int kFirst = 1 + kReducers;          // first workgroup with slots
  // The reducers and outlet blocks take the first hardware ids, which go to
  // the eight XCDs in turn; the bulk tiles after them are remapped so that
  // each XCD works on one contiguous range (nspecial is a multiple of 8).
  const int b = int(blockIdx.x);
  const int nb = L.nblocks - L.nspecial;
  const int v = b < L.nspecial ? b
                : L.nspecial + (L.xcd_chunk > 0 && LBM_XCD_REMAP
                                    ? xcd_remap_chunks(b - L.nspecial, nb, L.xcd_chunk)
                                    : xcd_remap(b - L.nspecial, nb));
  if (v < kFirst) {
    if (v == 0) {
      if (L.reduce2) reduce_level2(L.lvl_r, L);
    } else if (L.reduce1) {
      reduce_level1(static_cast<const T*>(L.part_r), v - 1, L);
    }
    return;
  }
  T* part = static_cast<T*>(L.part_w) + kPartials * kWaves * (v - kFirst);
  if constexpr (OUT != 0) {
    if (v < kFirst + L.n_nn) {
      if constexpr (OUT == OUTLET_CBC) {
        __shared__ CbcSmem<T> sm;
        cbc_block<S, MRT>(L, v - kFirst, sm, part);
      } else {
        __shared__ NnSmem<T> sm;
        nn_block<S, MRT>(L, v - kFirst, sm, part);
      }
      return;
    }
  }
  if (v < L.nspecial) {                          // padding: empty slots
    wave_partials(T(0), T(0), T(0), T(0), part);
    return;
  }
  bulk_block<S, MRT, PATH>(L, v - L.nspecial, part);
}

// Flush the pipeline after the last step: level 2 of the step before, then
// the last step's slots in one workgroup.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_finalize(const StepLaunch L) {
  if (L.reduce2) reduce_level2(L.lvl_r, L);
  __syncthreads();
  if (L.reduce1) {
    double t[4];
    sum_slots(static_cast<const T*>(L.part_r), 0, L.nslots, t);
    if (threadIdx.x == 0) commit_step(t, L);
  }
}

template <typename S, int MRT, int OUT>
static void launch_path(const StepLaunch& L, hipStream_t s) {
  if (L.path == PATH_VECTOR)
    hipLaunchKernelGGL((k_step<S, MRT, OUT, PATH_VECTOR>), dim3(L.nblocks), dim3(kBlock), 0, s, L);
  else
    hipLaunchKernelGGL((k_step<S, MRT, OUT, PATH_SCALAR>), dim3(L.nblocks), dim3(kBlock), 0, s, L);
}

template <typename S, int MRT>
static hipError_t launch_step_t(const StepLaunch& L, hipStream_t s) {
  if (!L.n_nn)
    launch_path<S, MRT, 0>(L, s);
  else if (L.outlet == OUTLET_CBC)
    launch_path<S, MRT, OUTLET_CBC>(L, s);
  else
    launch_path<S, MRT, OUTLET_NN>(L, s);
  return hipGetLastError();
}

hipError_t launch_step(const StepLaunch& L, hipStream_t s) {
  switch (L.precision * 2 + L.collision) {
    case LBM_FP64 * 2 + LBM_BGK: return launch_step_t<double, 0>(L, s);
    case LBM_FP64 * 2 + LBM_MRT: return launch_step_t<double, 1>(L, s);
    case LBM_FP32_OFFSET * 2 + LBM_BGK: return launch_step_t<float, 0>(L, s);
    case LBM_FP32_OFFSET * 2 + LBM_MRT: return launch_step_t<float, 1>(L, s);
    case LBM_FP16_OFFSET * 2 + LBM_BGK: return launch_step_t<__half, 0>(L, s);
    case LBM_FP16_OFFSET * 2 + LBM_MRT: return launch_step_t<__half, 1>(L, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const StepLaunch& L, hipStream_t s) {
  if (L.precision == LBM_FP64)
    hipLaunchKernelGGL((k_finalize<double>), dim3(1), dim3(kBlock), 0, s, L);
  else
    hipLaunchKernelGGL((k_finalize<float>), dim3(1), dim3(kBlock), 0, s, L);
  return hipGetLastError();
}

// ---- two steps per launch (Zou & He outflow) --------------------------------------
// Every wave owns a strip of kPairCols columns and pair_rows rows and takes
// both steps t+1 and t+2 of it in registers: lane l holds column x0 - 2 + l
// and walks down rows y0 - 2 .. y0 + pair_rows + 1, keeping the last three
// rows as read (step t) and the last three rows after the first collision
// (step t+1); each node pulls from the rows above and below in its window
// and from the neighbouring columns by lane shuffles, so a pair of steps
// reads and writes each population once (plus the strip's two-column and
// two-row halo, recomputed by the neighbouring strips).  Lanes 2..61 write
// step t+2.  The node code is the single-step one (bounce-back by the link
// word, Zou & He columns, force and mass of every fluid node, collision), so
// the populations are those of two single steps.  Per step and wave one
// partial slot (FP64 whatever the storage); the next launch's reducers take
// both steps (level 1), the one after commits them in order (level 2), as
// for single steps.
constexpr int kPairCols = 60;          // output columns per wave
constexpr int kPairRowsMin = 12, kPairRowsMax = 18;   // strip heights (pair_rows)

// The value of the lane to the left (lane - 1) or right (lane + 1) by a
// whole-wave DPP shift (a VALU move; lanes 0 and 63 get no neighbour and are
// halo lanes here).  bound_ctrl writes zero into those lanes, so no lane
// keeps the destination's old value and no move sets it up first (six
// moves fewer per step of a strip row, about 1 % of a launch).
template <int DIR>
__device__ __forceinline__ int lane_shift(int v) {
  return __builtin_amdgcn_update_dpp(0, v, DIR > 0 ? 0x138 : 0x130, 0xF, 0xF, true);   // wave_shr:1 / wave_shl:1
}
template <int DIR>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(float, lane_shift<DIR>(__builtin_bit_cast(int, v)));
}
template <int DIR>
__device__ __forceinline__ double lane_shift(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = lane_shift<DIR>(int(b & 0xFFFFFFFFll)), hi = lane_shift<DIR>(int(b >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) |
                                        static_cast<long long>(static_cast<unsigned>(lo)));
}

template <typename T>
__device__ __forceinline__ void pair_pull(const T lo[9], const T mid[9], const T hi[9], T g[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const T v = cy(q) == 1 ? lo[q] : (cy(q) == -1 ? hi[q] : mid[q]);
    // population q comes from column x - c_x: the left lane for c_x = +1
    g[q] = cx(q) == 0 ? v : (cx(q) == 1 ? lane_shift<1>(v) : lane_shift<-1>(v));
  }
}

// One node update from its pulled populations g and its own row values
// `own` (the bounce-back sources); returns false for a solid node.
template <typename T, int MRT>
__device__ __forceinline__ bool pair_node(const StepLaunch& L, uint32_t lk, int y, const T own[9],
                                          T g[9], bool count, T& fx, T& fy, T& dm) {
  if (lk & LINK_SOLID) return false;
  // bounce-back as selects: a branch per direction here made the compiler
  // keep g in scratch memory (77 instead of 53 us per step at 4096 x 1024)
#pragma unroll
  for (int q = 1; q < 9; ++q) g[q] = ((lk >> q) & 1u) ? own[opp(q)] : g[q];
  if (lk & LINK_INLET) {
    // the row's inlet velocity by a scalar load (y is wave-uniform), which
    // waits on its own counter rather than on the rows in flight
    using cp = const __attribute__((address_space(4))) double*;
    zouhe_inlet(g, L.inlet ? T(((cp)(L.inlet))[y]) : T(L.u_in));
  } else if (lk & LINK_OUTLET) {
    zouhe_outlet(g, T(L.one_minus_rho_out));
  }
  if (count) {
    add_force(lk, g, fx, fy);
    dm += macro(g).drho;
  }
  collide<T, MRT>(g, L);
  return true;
}

// The strip of wave `wave` and the column of this lane.
template <typename S>
struct PairWave {
  int lane, y0, ye, nrow;
  int xl, xs;              // this lane's column, and where it is read
  uint32_t off;            // byte offset of column xs within a row
  bool col_in, out_col;

  __device__ PairWave(const StepLaunch& L, int wave) {
    lane = threadIdx.x & 63;
    const int nstrip = (L.pair_nx + kPairCols - 1) / kPairCols;
    const int strip = wave % nstrip, seg = wave / nstrip;
    const int x0 = strip * kPairCols;
    y0 = seg * L.pair_rows;
    xl = x0 - 2 + lane;
    xs = xl;
    if (L.xper) xs = xs < 0 ? xs + L.nx : (xs >= L.nx ? xs - L.nx : xs);
    else xs = xs < 0 ? 0 : (xs >= L.nx ? L.nx - 1 : xs);
    off = uint32_t(xs) * uint32_t(sizeof(S));
    // a lattice node (periodic x: every lane, wrapped); the output columns
    // are the strip's own, unwrapped
    col_in = L.xper || (xl >= 0 && xl < L.nx);
    out_col = lane >= 2 && lane < 2 + kPairCols && xl < L.pair_nx;
    ye = min(y0 + L.pair_rows, L.ny);
    nrow = ye - y0 + 4;
  }

  __device__ int wrap_row(int y, const StepLaunch& L) const {
    if (L.yper) return y < 0 ? y + L.ny : (y >= L.ny ? y - L.ny : y);
    return y < 0 ? 0 : (y >= L.ny ? L.ny - 1 : y);
  }
};

// Strip `wave` of the bulk; its partials go to slot `slot`.
//
// The walk keeps three rows as read (R0..R2, step t), three rows after the
// first collision (S0..S2, step t+1) and the next row's loads (P).  Row j
// is fetched at the top of iteration j - 1 and copied into R2 at the top of
// iteration j.  In the plain walk (HOLD = 0) the fetch reads the row's
// link-chunk flag and branches on it, and loads and stores share one
// completion counter, so that wait also waits for the row's own loads and
// for the stores before them: a wave's loads overlap other waves' work
// only.  The held walk (HOLD = 1) reads the flags of the whole strip first
// and issues a row's stores one row late, with the next row's loads; its
// one wait per row then comes after the row's work (pair_hold chooses).
// Measured alternatives at 4096 x 1024 FP32 with 24-row strips, in the
// plain walk (not kept): fetching one row further ahead (-4 %), rings of 4
// to 6 rows unrolled in registers (-8 to -17 %), one scalar flag load per
// row (-2 %), a separate path for rows without link words (-4 %; +6 % at
// 16384 x 4096), FP32 sums of the strip's force terms (+1 %).  The strip
// height is chosen per lattice (pair_rows).  Loads and stores take the default cache policy: the
// strips' halo rows and their partly shared 128-byte lines are then found
// in the caches (non-temporal loads and stores: 88 against 100 thousand
// MLUPS at 4096 x 1024 and 78 against 107 at 16384 x 4096; non-temporal
// stores alone were 3 % faster at 4096 x 1024 FP32 only and 5-16 % slower
// at FP16 and FP64 and at 4096 x 2048, 8192 x 2048 and 16384 x 4096).
template <typename S, int MRT, int HOLD>
__device__ __forceinline__ void pair_strip(const StepLaunch& L, int wave, int slot, double* part) {
  using T = typename Store<S>::T;
  const PairWave<S> w(L, wave);
  const int y0 = w.y0, ye = w.ye, nrow = w.nrow;
  const bool col_in = w.col_in, out_col = w.out_col;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  T R0[9], R1[9], R2[9], S0[9], S1[9], S2[9], P[9];
  uint32_t K0 = 0, K1 = 0, K2 = 0, KP = 0;
  double fxa = 0.0, fya = 0.0, dma = 0.0, fxb = 0.0, fyb = 0.0, dmb = 0.0;
  // HOLD: bit j of lmask says that row y0 - 2 + j is a lattice row whose
  // 256-column chunk at this lane's column holds link words.  All flags are
  // loaded here at once, so that no load of the row walk waits on another
  // and the loads of a row are waited for only after the row's work.
  static_assert(kPairRowsMax + 4 <= 32, "one flag bit per strip row");
  uint32_t lmask = 0;
  if constexpr (HOLD) {
    uint8_t fl[kPairRowsMax + 4];
#pragma unroll
    for (int j = 0; j < kPairRowsMax + 4; ++j) {
      const int yr = y0 - 2 + j;
      const bool row_in = L.yper || (yr >= 0 && yr < L.ny);
      fl[j] = (j < nrow && row_in && col_in) ? L.chunk[w.wrap_row(yr, L) * L.nchunk + w.xs / kChunk]
                                              : uint8_t(0);
    }
#pragma unroll
    for (int j = 0; j < kPairRowsMax + 4; ++j) lmask |= uint32_t(fl[j] != 0) << j;
  }
  // row yr (absolute, may lie outside) into P and its link words into KP
  // (where the row's 256-column chunk has any)
  auto fetch = [&](int yr) {
    const int ys = w.wrap_row(yr, L);
    const int64_t row = int64_t(ys) * L.pitch;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      P[q] = Store<S>::ld(reinterpret_cast<const S*>(
          reinterpret_cast<const char*>(A + int64_t(q) * L.plane + row) + w.off));
    }
    KP = 0;
    if constexpr (HOLD) {
      if ((lmask >> (yr - (y0 - 2))) & 1u) KP = L.links[row + w.xs];
    } else {
      const bool row_in = L.yper || (yr >= 0 && yr < L.ny);
      if (row_in && col_in && L.chunk[ys * L.nchunk + w.xs / kChunk]) KP = L.links[row + w.xs];
    }
  };
  // HOLD: the step-(t+2) values of a row (H, at byte offset oh) are stored
  // with the next row's loads, so that both have that row's work to finish
  T H[9];
  uint32_t oh = 0;
  bool held = false;
  auto flush = [&]() {
    if (held) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
        Store<S>::st_cached(reinterpret_cast<S*>(reinterpret_cast<char*>(B + int64_t(q) * L.plane) + oh),
                            H[q]);
    }
    held = false;
  };
  fetch(y0 - 2);
  for (int j = 0; j < nrow; ++j) {
    const int yr = y0 - 2 + j;
#pragma unroll
    for (int q = 0; q < 9; ++q) R2[q] = P[q];
    K2 = KP;
    if (j + 1 < nrow) fetch(yr + 1);
    if constexpr (HOLD) flush();
    if (j >= 2) {
      // step t+1 at row yr - 1 from rows yr-2 .. yr
      const int y1 = yr - 1;
      const bool in1 = L.yper || (y1 >= 0 && y1 < L.ny);
      const bool cnt1 = out_col && y1 >= y0 && y1 < ye;
      T g[9];
      pair_pull(R0, R1, R2, g);
      T fx1 = T(0), fy1 = T(0), dm1 = T(0);
      if (!(in1 && col_in && pair_node<T, MRT>(L, K1, w.wrap_row(y1, L), R1, g, cnt1, fx1, fy1, dm1))) {
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = R1[q];   // solid or outside: unchanged
      }
      fxa += double(fx1);
      fya += double(fy1);
      dma += double(dm1);
      // the state of step t+1 as a store and reload would give it (FP16
      // storage rounds here, as one launch per step does)
#pragma unroll
      for (int q = 0; q < 9; ++q) S2[q] = Store<S>::stored(g[q]);
      if (j >= 4) {
        // step t+2 at row yr - 2 (always one of the strip's rows) from the
        // step-(t+1) rows yr-3 .. yr-1
        const int y2 = yr - 2;
        pair_pull(S0, S1, S2, g);
        const uint32_t o2 = uint32_t(y2) * uint32_t(L.pitch) * uint32_t(sizeof(S)) + w.off;
        T fx2 = T(0), fy2 = T(0), dm2 = T(0);
        if (out_col && pair_node<T, MRT>(L, K0, y2, S1, g, true, fx2, fy2, dm2)) {
          if constexpr (HOLD) {
#pragma unroll
            for (int q = 0; q < 9; ++q) H[q] = g[q];
            oh = o2;
            held = true;
          } else {
#pragma unroll
            for (int q = 0; q < 9; ++q)
              Store<S>::st_cached(
                  reinterpret_cast<S*>(reinterpret_cast<char*>(B + int64_t(q) * L.plane) + o2), g[q]);
          }
        }
        fxb += double(fx2);
        fyb += double(fy2);
        dmb += double(dm2);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        S0[q] = S1[q];
        S1[q] = S2[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      R0[q] = R1[q];
      R1[q] = R2[q];
    }
    K0 = K1;
    K1 = K2;
  }
  if constexpr (HOLD) flush();
  // one slot per wave and step: [0, n) the first step, [n, 2n) the second
  const int n = L.pair_nslots;
  fxa = wave_sum(fxa); fya = wave_sum(fya); dma = wave_sum(dma);
  fxb = wave_sum(fxb); fyb = wave_sum(fyb); dmb = wave_sum(dmb);
  if (w.lane == 0) {
    double* a = part + int64_t(kPartials) * slot;
    double* b = part + int64_t(kPartials) * (n + slot);
    a[0] = fxa; a[1] = fya; a[2] = dma; a[3] = 0.0;
    b[0] = fxb; b[1] = fyb; b[2] = dmb; b[3] = 0.0;
  }
}

// ---- two steps per launch at the neural outlet (Sec. 3.1, Eq. 16) -------------
// An outlet block takes both steps of the last kOutCols columns (nx-4 .. nx-1)
// for kOutRows rows y0 .. y0+61; the bulk strips stop at column nx-5.  It
// stages A_t over columns nx-6 .. nx-1 and rows y0-2 .. y0+63, takes step t+1
// on columns nx-5 .. nx-1 for rows y0-1 .. y0+62 -- the outlet column
// through the network on those 64 rows -- then step t+2 on its own columns
// and rows, the network on its 62 rows.  Every node runs the single-step
// node code (pull with bounce-back by the link word, force and mass, Eq. 16
// with its fallback, collision), and the state between the steps is rounded
// as a store would round it, so the result is that of two single steps.
constexpr int kOutCols = 4;                 // columns nx-4 .. nx-1
constexpr int kOutRows = kNnRows - 2;       // rows per outlet block
constexpr int kSt2Rows = kOutRows + 4;      // staged rows y0-2 .. y0+63
constexpr int kSt2Cols = kOutCols + 2;      // staged columns nx-6 .. nx-1
constexpr int kS1Rows = kOutRows + 2;       // step t+1 rows y0-1 .. y0+62
constexpr int kS1Cols = kOutCols + 1;       // step t+1 columns nx-5 .. nx-1
static_assert(kS1Rows == kNnRows && kBlock == 4 * kNnRows, "one network tile per step");

template <typename T>
struct alignas(16) Nn2Smem {
  union {
    T st[9 * kSt2Rows * kSt2Cols];   // A_t (dead once step t+1 has pulled it)
    MlpH H;                          // network activations
  } u;
  T s1[9 * kS1Rows * kS1Cols];       // post-collision state of step t+1
  MlpX X;
  T prev[kNnRows * 4];               // g3, g6, g7, density offset at x = L-1
};

// Row y of the lattice for a block row (periodic wrap, or -1 outside walls).
// A block's rows reach y0 + 63, more than one period when ny < 64.
__device__ __forceinline__ int block_row(const StepLaunch& L, int y) {
  if (L.yper) return ((y % L.ny) + L.ny) % L.ny;
  return (y < 0 || y >= L.ny) ? -1 : y;
}

// Pull the populations of node (r, c) of a staged tile src[q][R][C] (row
// and column of the tile), bounce-back by the link word from the node's own
// values.  Unknowns of the outlet column (source beyond the last staged
// column) get the node's own value, replaced later.
template <typename T, int R, int C>
__device__ __forceinline__ void tile_pull(const T* src, int r, int c, uint32_t lk, T g[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const bool bb = (lk >> q) & 1u;
    const int cc = bb ? c : c - cx(q);
    const bool out = cc >= C;
    const int qq = (bb || out) ? opp(q) : q;
    g[q] = src[(qq * R + ((bb || out) ? r : r - cy(q))) * C + (out ? c : cc)];
  }
}

template <typename S, int MRT>
__device__ void nn2_block(const StepLaunch& L, int nb, Nn2Smem<typename Store<S>::T>& sm,
                          double* part, int slot) {
  using T = typename Store<S>::T;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const MlpDev* __restrict__ w = L.mlp;
  const int y0 = nb * kOutRows;
  const int xs0 = L.nx - kSt2Cols;           // first staged column
  const int tid = threadIdx.x;
  const int j = tid & 63, k = tid >> 6;
  double fx1 = 0, fy1 = 0, dm1 = 0, nf1 = 0, fx2 = 0, fy2 = 0, dm2 = 0, nf2 = 0;

  // 1. stage A_t[q][y0-2 .. y0+63][nx-6 .. nx-1]
  for (int i = tid; i < 9 * kSt2Rows * kSt2Cols; i += kBlock) {
    const int q = i / (kSt2Rows * kSt2Cols);
    const int rem = i - q * (kSt2Rows * kSt2Cols);
    const int r = rem / kSt2Cols, c = rem - r * kSt2Cols;
    int y = y0 - 2 + r;
    y = L.yper ? (y + 2 * L.ny) % L.ny : min(max(y, 0), L.ny - 1);   // clamped rows: never pulled
    sm.u.st[i] = Store<S>::ld(A + int64_t(q) * L.plane + int64_t(y) * L.pitch + xs0 + c);
  }
  __syncthreads();

  // 2. step t+1 on columns nx-5 .. nx-2 (thread: row y0-1+j, column nx-5+k),
  // and the pull of the outlet column (threads k = 0)
  {
    const int yb = block_row(L, y0 - 1 + j);
    const int x = L.nx - 5 + k;
    const uint32_t lk = yb >= 0 ? L.links[int64_t(yb) * L.pitch + x] : LINK_SOLID;
    const bool own = j >= 1 && j <= kOutRows && y0 - 1 + j < L.ny;   // the block's own rows
    T g[9];
    tile_pull<T, kSt2Rows, kSt2Cols>(sm.u.st, j + 1, k + 1, lk, g);
    const bool live = !(lk & LINK_SOLID);
    if (k >= 1) {
      // features of column x = L-1-jc, feature index 9 jc + q
      const int jc = 3 - k;
#pragma unroll
      for (int q = 0; q < 9; ++q)
        sm.X.x[j * kXPitch + 9 * jc + q] = live ? feature_bf16(w, 9 * jc + q, float(g[q])) : 0;
      if (k == 3) {
        sm.prev[j * 4 + 0] = g[3];
        sm.prev[j * 4 + 1] = g[6];
        sm.prev[j * 4 + 2] = g[7];
        sm.prev[j * 4 + 3] = macro(g).drho;
      }
    } else {
#pragma unroll
      for (int f = 27; f < 32; ++f) sm.X.x[j * kXPitch + f] = 0;
    }
    if (live) {
      if (own && k >= 1) {
        T fx = T(0), fy = T(0);
        add_force(lk, g, fx, fy);
        fx1 += double(fx);
        fy1 += double(fy);
        dm1 += double(macro(g).drho);
      }
      collide<T, MRT>(g, L);
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) g[q] = sm.u.st[(q * kSt2Rows + j + 1) * kSt2Cols + k + 1];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) sm.s1[(q * kS1Rows + j) * kS1Cols + k] = Store<S>::stored(g[q]);
  }
  // the outlet node of row y0-1+j at step t+1: its known populations now
  uint32_t lko = LINK_SOLID;
  T go[9];
  if (k == 0) {
    const int yb = block_row(L, y0 - 1 + j);
    lko = yb >= 0 ? L.links[int64_t(yb) * L.pitch + L.nx - 1] : LINK_SOLID;
    tile_pull<T, kSt2Rows, kSt2Cols>(sm.u.st, j + 1, kSt2Cols - 1, lko, go);
    if (lko & LINK_SOLID) {
#pragma unroll
      for (int q = 0; q < 9; ++q) go[q] = sm.u.st[(q * kSt2Rows + j + 1) * kSt2Cols + kSt2Cols - 1];
    }
  }
  __syncthreads();                      // features, prev; the stage is dead
  mlp_tile(w, sm.X, sm.u.H);
  if (k == 0) {
    const bool own = j >= 1 && j <= kOutRows && y0 - 1 + j < L.ny;
    if (!(lko & LINK_SOLID)) {
      T fx = T(0), fy = T(0);
      if (own) add_force(lko, go, fx, fy);
      const bool kept = nn_reconstruct(w, &sm.u.H.o[j * 4], &sm.prev[j * 4], go,
                                       T(L.one_minus_rho_out));
      if (own) {
        fx1 += double(fx);
        fy1 += double(fy);
        dm1 += double(macro(go).drho);
        nf1 += kept ? 0.0 : 1.0;
      }
      collide<T, MRT>(go, L);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) sm.s1[(q * kS1Rows + j) * kS1Cols + kS1Cols - 1] = Store<S>::stored(go[q]);
  }
  __syncthreads();                      // s1 complete; H read

  // 3. step t+2 on the block's own rows y0 + j (j < 62): columns nx-4 .. nx-2
  // (k = 0 .. 2), the outlet column (k = 3)
  const int y = y0 + j;
  const bool row_ok = j < kOutRows && y < L.ny;
  const uint32_t lk = row_ok ? L.links[int64_t(y) * L.pitch + L.nx - 4 + k] : LINK_SOLID;
  T g[9];
  // rows j >= kOutRows are no output rows: their (unused) pull stays inside s1
  tile_pull<T, kS1Rows, kS1Cols>(sm.s1, min(j, kOutRows - 1) + 1, k + 1, lk, g);
  const bool live = row_ok && !(lk & LINK_SOLID);
  if (k < 3) {
    const int jc = 2 - k;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      sm.X.x[j * kXPitch + 9 * jc + q] = live ? feature_bf16(w, 9 * jc + q, float(g[q])) : 0;
    if (k == 2) {
      sm.prev[j * 4 + 0] = g[3];
      sm.prev[j * 4 + 1] = g[6];
      sm.prev[j * 4 + 2] = g[7];
      sm.prev[j * 4 + 3] = macro(g).drho;
    }
    if (live) {
      T fx = T(0), fy = T(0);
      add_force(lk, g, fx, fy);
      fx2 += double(fx);
      fy2 += double(fy);
      dm2 += double(macro(g).drho);
      collide<T, MRT>(g, L);
      const int64_t row = int64_t(y) * L.pitch + L.nx - 4 + k;
#pragma unroll
      for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row, g[q]);
    }
  } else {
#pragma unroll
    for (int f = 27; f < 32; ++f) sm.X.x[j * kXPitch + f] = 0;
  }
  __syncthreads();
  mlp_tile(w, sm.X, sm.u.H);
  if (k == 3 && live) {
    T fx = T(0), fy = T(0);
    add_force(lk, g, fx, fy);
    const bool kept = nn_reconstruct(w, &sm.u.H.o[j * 4], &sm.prev[j * 4], g,
                                     T(L.one_minus_rho_out));
    fx2 += double(fx);
    fy2 += double(fy);
    dm2 += double(macro(g).drho);
    nf2 += kept ? 0.0 : 1.0;
    collide<T, MRT>(g, L);
    const int64_t row = int64_t(y) * L.pitch + L.nx - 1;
#pragma unroll
    for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row, g[q]);
  }
  // one slot per wave and step, as the strips
  const int n = L.pair_nslots;
  fx1 = wave_sum(fx1); fy1 = wave_sum(fy1); dm1 = wave_sum(dm1); nf1 = wave_sum(nf1);
  fx2 = wave_sum(fx2); fy2 = wave_sum(fy2); dm2 = wave_sum(dm2); nf2 = wave_sum(nf2);
  if (j == 0) {
    double* a = part + int64_t(kPartials) * (slot + k);
    double* b = part + int64_t(kPartials) * (n + slot + k);
    a[0] = fx1; a[1] = fy1; a[2] = dm1; a[3] = nf1;
    b[0] = fx2; b[1] = fy2; b[2] = dm2; b[3] = nf2;
  }
}

// ---- two steps per launch at the characteristic outlet (Sec. 4) ----------------
// The geometry of the neural outlet blocks: own columns nx-4 .. nx-1 and 62
// rows, A_t staged over columns nx-6 .. nx-1 and rows y0-2 .. y0+63.  Step
// t+1 runs on columns nx-5 .. nx-1 for rows y0-1 .. y0+62, the outlet column
// from the LODI update of the moments of A_t; step t+2 on the own columns
// and rows from the moments of the step-(t+1) state, the network features
// taking the time derivatives of step t+1 from LDS.  The time derivatives
// are read from L.cbc_dt (rows of step t) and written to L.cbc_dt_w (own
// rows of step t+2): neighbouring blocks read the rows this block writes.
// Periodic laterals (the library rejects walls for this outflow).
template <typename T>
struct alignas(16) Cbc2Smem {
  T st[9 * kSt2Rows * kSt2Cols];     // A_t
  T s1[9 * kS1Rows * kS1Cols];       // post-collision state of step t+1
  T mo[3 * 3 * kSt2Rows];            // moments of columns nx-3 .. nx-1 (step t, then t+1)
  T dt1[kNnRows * 3];                // p_t, u_t, v_t of step t+1 per step-(t+1) row
  CbcNetSmem<T> net;
};

template <typename S, int MRT>
__device__ void cbc2_block(const StepLaunch& L, int nb, Cbc2Smem<typename Store<S>::T>& sm,
                           double* part, int slot) {
  using T = typename Store<S>::T;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const CbcDev* __restrict__ c = L.cbc;
  const int y0 = nb * kOutRows;
  const int xs0 = L.nx - kSt2Cols;
  const int tid = threadIdx.x;
  const int j = tid & 63, k = tid >> 6;
  double fx1 = 0, fy1 = 0, dm1 = 0, fx2 = 0, fy2 = 0, dm2 = 0;

  // 1. stage A_t[q][y0-2 .. y0+63][nx-6 .. nx-1] (rows wrapped)
  for (int i = tid; i < 9 * kSt2Rows * kSt2Cols; i += kBlock) {
    const int q = i / (kSt2Rows * kSt2Cols);
    const int rem = i - q * (kSt2Rows * kSt2Cols);
    const int r = rem / kSt2Cols, cc = rem - r * kSt2Cols;
    const int y = (y0 - 2 + r + 2 * L.ny) % L.ny;
    sm.st[i] = Store<S>::ld(A + int64_t(q) * L.plane + int64_t(y) * L.pitch + xs0 + cc);
  }
  __syncthreads();
  tile_moments<T, kSt2Rows, kSt2Cols>(sm.st, kSt2Cols - 3, sm.mo);

  // 2. step t+1 on columns nx-5 .. nx-2 (thread: row y0-1+j, column nx-5+k)
  {
    const int yb = (y0 - 1 + j + L.ny) % L.ny;
    const int x = L.nx - 5 + k;
    const uint32_t lk = L.links[int64_t(yb) * L.pitch + x];
    const bool own = j >= 1 && j <= kOutRows && y0 - 1 + j < L.ny;
    T g[9];
    tile_pull<T, kSt2Rows, kSt2Cols>(sm.st, j + 1, k + 1, lk, g);
    if (!(lk & LINK_SOLID)) {
      if (own && k >= 1) {
        T fx = T(0), fy = T(0);
        add_force(lk, g, fx, fy);
        fx1 += double(fx);
        fy1 += double(fy);
        dm1 += double(macro(g).drho);
      }
      collide<T, MRT>(g, L);
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) g[q] = sm.st[(q * kSt2Rows + j + 1) * kSt2Cols + k + 1];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) sm.s1[(q * kS1Rows + j) * kS1Cols + k] = Store<S>::stored(g[q]);
  }
  __syncthreads();                      // moments of A_t
  // the outlet column at step t+1, rows y0-1+j (thread j < 64)
  T sigma = T(c->sigma), kappa2 = T(c->kappa2);
  {
    const int yb = (y0 - 1 + j + L.ny) % L.ny;
    if (c->has_net) {
      if (tid < kNnRows) {
        T g6[6];
        cbc_gradients<T, kSt2Rows>(sm.mo, j + 1, g6);
        const double* d = L.cbc_dt + 4 * int64_t(yb);
        const T prev[3] = {T(d[0]), T(d[1]), T(d[2])};
        cbc_features(c, g6, prev, &sm.net.feat[j * kCbcIn]);
      }
      cbc_network(c, sm.net, sigma, kappa2);
    }
    if (tid < kNnRows) {
      const uint32_t lk = L.links[int64_t(yb) * L.pitch + L.nx - 1];
      const bool own = j >= 1 && j <= kOutRows && y0 - 1 + j < L.ny;
      T g[9];
      tile_pull<T, kSt2Rows, kSt2Cols>(sm.st, j + 1, kSt2Cols - 1, lk, g);
      if (!(lk & LINK_SOLID)) {
        const int r = j + 1;
        T g6[6], nst[3], dt[3];
        cbc_gradients<T, kSt2Rows>(sm.mo, r, g6);
        cbc_lodi(c, g6, sm.mo[(0 * 3 + 2) * kSt2Rows + r], sm.mo[(1 * 3 + 2) * kSt2Rows + r],
                 sm.mo[(2 * 3 + 2) * kSt2Rows + r], sigma, kappa2, nst, dt);
        sm.dt1[j * 3 + 0] = dt[0];
        sm.dt1[j * 3 + 1] = dt[1];
        sm.dt1[j * 3 + 2] = dt[2];
        outlet_state(g, nst[0], nst[1], nst[2]);
        if (own) {
          T fx = T(0), fy = T(0);
          add_force(lk, g, fx, fy);
          fx1 += double(fx);
          fy1 += double(fy);
          dm1 += double(macro(g).drho);
        }
        collide<T, MRT>(g, L);
      } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = sm.st[(q * kSt2Rows + j + 1) * kSt2Cols + kSt2Cols - 1];
        sm.dt1[j * 3 + 0] = sm.dt1[j * 3 + 1] = sm.dt1[j * 3 + 2] = T(0);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q)
        sm.s1[(q * kS1Rows + j) * kS1Cols + kS1Cols - 1] = Store<S>::stored(g[q]);
    }
  }
  __syncthreads();                      // s1 complete
  // moments of the step-(t+1) state at columns nx-3 .. nx-1, rows y0-1 .. y0+62
  tile_moments<T, kS1Rows, kS1Cols>(sm.s1, kS1Cols - 3, sm.mo);

  // 3. step t+2 on the own rows y0 + j (j < 62): columns nx-4 .. nx-2 (k < 3)
  const int y = y0 + j;
  const bool row_ok = j < kOutRows && y < L.ny;
  if (k < 3 && row_ok) {
    const uint32_t lk = L.links[int64_t(y) * L.pitch + L.nx - 4 + k];
    if (!(lk & LINK_SOLID)) {
      T g[9];
      tile_pull<T, kS1Rows, kS1Cols>(sm.s1, j + 1, k + 1, lk, g);
      T fx = T(0), fy = T(0);
      add_force(lk, g, fx, fy);
      fx2 += double(fx);
      fy2 += double(fy);
      dm2 += double(macro(g).drho);
      collide<T, MRT>(g, L);
      const int64_t off = int64_t(y) * L.pitch + L.nx - 4 + k;
#pragma unroll
      for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + off, g[q]);
    }
  }
  __syncthreads();                      // moments of step t+1
  sigma = T(c->sigma);
  kappa2 = T(c->kappa2);
  if (c->has_net) {
    if (tid < kNnRows) {
      const int r = min(j, kOutRows - 1) + 1;    // rows j >= 62: unused
      T g6[6];
      cbc_gradients<T, kS1Rows>(sm.mo, r, g6);
      const T prev[3] = {sm.dt1[r * 3 + 0], sm.dt1[r * 3 + 1], sm.dt1[r * 3 + 2]};
      cbc_features(c, g6, prev, &sm.net.feat[j * kCbcIn]);
    }
    cbc_network(c, sm.net, sigma, kappa2);
  }
  if (tid < kNnRows && row_ok) {
    const uint32_t lk = L.links[int64_t(y) * L.pitch + L.nx - 1];
    if (!(lk & LINK_SOLID)) {
      const int r = j + 1;
      T g[9], g6[6], nst[3], dt[3];
      tile_pull<T, kS1Rows, kS1Cols>(sm.s1, r, kS1Cols - 1, lk, g);
      cbc_gradients<T, kS1Rows>(sm.mo, r, g6);
      cbc_lodi(c, g6, sm.mo[(0 * 3 + 2) * kS1Rows + r], sm.mo[(1 * 3 + 2) * kS1Rows + r],
               sm.mo[(2 * 3 + 2) * kS1Rows + r], sigma, kappa2, nst, dt);
      double* d = L.cbc_dt_w + 4 * int64_t(y);
      d[0] = double(dt[0]);
      d[1] = double(dt[1]);
      d[2] = double(dt[2]);
      outlet_state(g, nst[0], nst[1], nst[2]);
      T fx = T(0), fy = T(0);
      add_force(lk, g, fx, fy);
      fx2 += double(fx);
      fy2 += double(fy);
      dm2 += double(macro(g).drho);
      collide<T, MRT>(g, L);
      const int64_t off = int64_t(y) * L.pitch + L.nx - 1;
#pragma unroll
      for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + off, g[q]);
    } else {
      double* d = L.cbc_dt_w + 4 * int64_t(y);
      d[0] = d[1] = d[2] = 0.0;
    }
  }
  const int n = L.pair_nslots;
  fx1 = wave_sum(fx1); fy1 = wave_sum(fy1); dm1 = wave_sum(dm1);
  fx2 = wave_sum(fx2); fy2 = wave_sum(fy2); dm2 = wave_sum(dm2);
  if (j == 0) {
    double* a = part + int64_t(kPartials) * (slot + k);
    double* b = part + int64_t(kPartials) * (n + slot + k);
    a[0] = fx1; a[1] = fy1; a[2] = dm1; a[3] = 0.0;
    b[0] = fx2; b[1] = fy2; b[2] = dm2; b[3] = 0.0;
  }
}

// Level 2 of a launch of K steps: each step's kReducers sums, committed in
// step order.
template <int K>
__device__ void multi_level2(const double* __restrict__ lvl, const StepLaunch& L) {
  for (int h = 0; h < K; ++h) {
    double s[4] = {0.0, 0.0, 0.0, 0.0}, t[4];
    if (threadIdx.x < kReducers) {
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] = lvl[(h * kReducers + threadIdx.x) * 4 + k];
    }
    block_sum4(s, t);
    if (threadIdx.x == 0) commit_step(t, L);
    __syncthreads();
  }
}

// Level 1 of a launch of K steps (n slots per step): reducer r (of
// K kReducers) sums its slice of one step's slots.
template <typename T>
__device__ void multi_level1(const T* __restrict__ part, int r, int n, const StepLaunch& L) {
  const int h = r / kReducers, rr = r - h * kReducers;
  const int per = (n + kReducers - 1) / kReducers;
  const int b0 = min(rr * per, n), b1 = min(b0 + per, n);
  double t[4];
  sum_slots(part + int64_t(kPartials) * h * n, b0, b1, t);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) L.lvl_w[(h * kReducers + rr) * 4 + k] = t[k];
  }
}

constexpr int kPairSpecial = (1 + 2 * kReducers + 7) / 8 * 8;

// OUT: 0 the Zou & He outlet inside the strips; OUTLET_NN or OUTLET_CBC the
// outlet blocks of the neural or characteristic outflow (the first pair_out
// workgroups after the reducers).
template <typename S, int MRT, int OUT, int HOLD>
__global__ void __launch_bounds__(kBlock) k_step2(const StepLaunch L) {
  const int v = int(blockIdx.x);
  if (v < kPairSpecial) {
    if (v == 0) {
      if (L.reduce2) multi_level2<2>(L.lvl_r, L);
    } else if (v <= 2 * kReducers && L.reduce1) {
      multi_level1(static_cast<const double*>(L.part_r), v - 1, L.pair_nslots, L);
    }
    return;
  }
  const int b = v - kPairSpecial;
  double* part = static_cast<double*>(L.part_w);
  if constexpr (OUT == OUTLET_NN) {
    if (b < L.pair_out) {
      __shared__ Nn2Smem<typename Store<S>::T> sm;
      nn2_block<S, MRT>(L, b, sm, part, b * kWaves);
      return;
    }
  } else if constexpr (OUT == OUTLET_CBC) {
    if (b < L.pair_out) {
      __shared__ Cbc2Smem<typename Store<S>::T> sm;
      cbc2_block<S, MRT>(L, b, sm, part, b * kWaves);
      return;
    }
  }
  // strip workgroups dealt to the XCDs: chunks of pair_chunk workgroups in
  // turn, or one contiguous eighth per XCD (pair_chunk 0)
  int sb = b - L.pair_out;
  const int nsb = int(gridDim.x) - kPairSpecial - L.pair_out;
  sb = L.pair_chunk > 0 ? xcd_remap_chunks(sb, nsb, L.pair_chunk) : xcd_remap(sb, nsb);
  // the wave's slot, held in a scalar register: the strip's rows and
  // columns are then wave-uniform values and its row addresses scalar
  const int slot = __builtin_amdgcn_readfirstlane((L.pair_out + sb) * kWaves + int(threadIdx.x >> 6));
  if (slot >= L.pair_nslots) return;                  // whole wave
  pair_strip<S, MRT, HOLD>(L, slot - L.pair_out * kWaves, slot, part);
}

// Flush after the last pair: level 2 of the pair before, then both steps of
// the last pair's slots in one workgroup.
// Flush after the last launch of K steps (n slots per step): level 2 of the
// launch before, then the K steps of the last launch's slots in one
// workgroup.
template <typename T, int K>
__global__ void __launch_bounds__(kBlock) k_finalize_multi(const StepLaunch L, int n) {
  if (L.reduce2) multi_level2<K>(L.lvl_r, L);
  __syncthreads();
  if (L.reduce1) {
    for (int h = 0; h < K; ++h) {
      double t[4];
      sum_slots(static_cast<const T*>(L.part_r) + int64_t(kPartials) * h * n, 0, n, t);
      if (threadIdx.x == 0) commit_step(t, L);
      __syncthreads();
    }
  }
}

template <typename S, int MRT, int HOLD>
static hipError_t launch_pair_h(const StepLaunch& L, hipStream_t s) {
  const int blocks = kPairSpecial + (L.pair_nslots + kWaves - 1) / kWaves;
  if (L.pair_out > 0 && L.outlet == OUTLET_NN)
    hipLaunchKernelGGL((k_step2<S, MRT, OUTLET_NN, HOLD>), dim3(blocks), dim3(kBlock), 0, s, L);
  else if (L.pair_out > 0 && L.outlet == OUTLET_CBC)
    hipLaunchKernelGGL((k_step2<S, MRT, OUTLET_CBC, HOLD>), dim3(blocks), dim3(kBlock), 0, s, L);
  else if (L.pair_out == 0)
    hipLaunchKernelGGL((k_step2<S, MRT, 0, HOLD>), dim3(blocks), dim3(kBlock), 0, s, L);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename S, int MRT>
static hipError_t launch_pair_t(const StepLaunch& L, hipStream_t s) {
  if constexpr (!std::is_same_v<S, __half>) {
    if (L.pair_hold) return launch_pair_h<S, MRT, 1>(L, s);
  }
  return L.pair_hold ? hipErrorInvalidValue : launch_pair_h<S, MRT, 0>(L, s);
}

// ---- three time steps per launch (Zou & He outflow) --------------------------------
//
// The two-step strip walk carried one step further: every wave owns a strip
// of kTriCols columns (lane l holds column x0 - 3 + l) and walks rows
// y0 - 3 .. y0 + rows + 2, keeping the last three rows as read (R), after
// the first collision (S) and after the second (U), and the next row's
// loads (P).  Step t+1 is taken on lanes 1..62 and rows y0 - 2 .. y0 + rows
// + 1, step t+2 on lanes 2..61 and rows y0 - 1 .. y0 + rows, step t+3 on the
// strip's own 58 columns and rows, which are stored.  The states after the
// first two steps are rounded to the storage precision as a store and
// reload would round them, so a launch equals three single launches bit for
// bit.  A launch reads and writes each population once for three steps:
// 24 B per node and step at FP32.  Each step's force and mass terms are
// summed over the nodes the strip owns (its columns and rows), FP64 per wave
// and step.
constexpr int kTriCols = 58;
constexpr int kTriRowsMax = 24;   // strip heights of the three-step walk (tri_rows)

template <typename S>
struct TriWave {
  int lane, y0, ye, nrow;
  int xl, xs;              // this lane's column, and where it is read
  uint32_t off;            // byte offset of column xs within a row
  bool col_in, out_col;

  __device__ TriWave(const StepLaunch& L, int wave) {
    lane = threadIdx.x & 63;
    const int nstrip = (L.tri_nx + kTriCols - 1) / kTriCols;
    const int strip = wave % nstrip, seg = wave / nstrip;
    const int x0 = strip * kTriCols;
    y0 = seg * L.tri_rows;
    xl = x0 - 3 + lane;
    xs = xl;
    if (L.xper) xs = xs < 0 ? xs + L.nx : (xs >= L.nx ? xs - L.nx : xs);
    else xs = xs < 0 ? 0 : (xs >= L.nx ? L.nx - 1 : xs);
    off = uint32_t(xs) * uint32_t(sizeof(S));
    col_in = L.xper || (xl >= 0 && xl < L.nx);
    out_col = lane >= 3 && lane < 3 + kTriCols && xl < L.tri_nx;
    ye = min(y0 + L.tri_rows, L.ny);
    nrow = ye - y0 + 6;
  }

  __device__ int wrap_row(int y, const StepLaunch& L) const {
    if (L.yper) return y < 0 ? y + L.ny : (y >= L.ny ? y - L.ny : y);
    return y < 0 ? 0 : (y >= L.ny ? L.ny - 1 : y);
  }
};

template <typename S, int MRT, int HOLD>
__device__ __forceinline__ void tri_strip(const StepLaunch& L, int wave, int slot, double* part) {
  using T = typename Store<S>::T;
  const TriWave<S> w(L, wave);
  const int y0 = w.y0, ye = w.ye, nrow = w.nrow;
  const bool col_in = w.col_in, out_col = w.out_col;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  T R0[9], R1[9], R2[9], S0[9], S1[9], S2[9], U0[9], U1[9], U2[9], P[9];
  // link words of rows yr - 3 (KM), yr - 2 (K0), yr - 1 (K1), yr (K2) and
  // the row being fetched (KP)
  uint32_t KM = 0, K0 = 0, K1 = 0, K2 = 0, KP = 0;
  double fx[3] = {0.0, 0.0, 0.0}, fy[3] = {0.0, 0.0, 0.0}, dm[3] = {0.0, 0.0, 0.0};
  // HOLD: the link-chunk flags of all the strip's rows first, and a row's
  // stores issued one row late (the held walk of pair_strip)
  static_assert(kTriRowsMax + 6 <= 32, "one flag bit per strip row");
  uint32_t lmask = 0;
  if constexpr (HOLD) {
    uint8_t fl[kTriRowsMax + 6];
#pragma unroll
    for (int jj = 0; jj < kTriRowsMax + 6; ++jj) {
      const int yr = y0 - 3 + jj;
      const bool row_in = L.yper || (yr >= 0 && yr < L.ny);
      fl[jj] = (jj < nrow && row_in && col_in) ? L.chunk[w.wrap_row(yr, L) * L.nchunk + w.xs / kChunk]
                                                : uint8_t(0);
    }
#pragma unroll
    for (int jj = 0; jj < kTriRowsMax + 6; ++jj) lmask |= uint32_t(fl[jj] != 0) << jj;
  }
  auto fetch = [&](int yr) {
    const int ys = w.wrap_row(yr, L);
    const int64_t row = int64_t(ys) * L.pitch;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      P[q] = Store<S>::ld(reinterpret_cast<const S*>(
          reinterpret_cast<const char*>(A + int64_t(q) * L.plane + row) + w.off));
    }
    KP = 0;
    if constexpr (HOLD) {
      if ((lmask >> (yr - (y0 - 3))) & 1u) KP = L.links[row + w.xs];
    } else {
      const bool row_in = L.yper || (yr >= 0 && yr < L.ny);
      if (row_in && col_in && L.chunk[ys * L.nchunk + w.xs / kChunk]) KP = L.links[row + w.xs];
    }
  };
  T H[9];
  uint32_t oh = 0;
  bool held = false;
  auto flush = [&]() {
    if (held) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
        Store<S>::st_cached(reinterpret_cast<S*>(reinterpret_cast<char*>(B + int64_t(q) * L.plane) + oh),
                            H[q]);
    }
    held = false;
  };
  // one intermediate step at row y (absolute) from the rows lo, mid, hi of
  // the state before it, own = mid; nodes outside the lattice, solid or in
  // a column outside keep their values
  auto inner = [&](const T lo[9], const T mid[9], const T hi[9], uint32_t lk, int y, int k, T out[9]) {
    const bool in = L.yper || (y >= 0 && y < L.ny);
    const bool cnt = out_col && y >= y0 && y < ye;
    T g[9];
    pair_pull(lo, mid, hi, g);
    T fxk = T(0), fyk = T(0), dmk = T(0);
    if (!(in && col_in && pair_node<T, MRT>(L, lk, w.wrap_row(y, L), mid, g, cnt, fxk, fyk, dmk))) {
#pragma unroll
      for (int q = 0; q < 9; ++q) g[q] = mid[q];
    }
    fx[k] += double(fxk);
    fy[k] += double(fyk);
    dm[k] += double(dmk);
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = Store<S>::stored(g[q]);
  };
  fetch(y0 - 3);
  for (int j = 0; j < nrow; ++j) {
    const int yr = y0 - 3 + j;
#pragma unroll
    for (int q = 0; q < 9; ++q) R2[q] = P[q];
    K2 = KP;
    if (j + 1 < nrow) fetch(yr + 1);
    if constexpr (HOLD) flush();
    if (j >= 2) {
      inner(R0, R1, R2, K1, yr - 1, 0, S2);               // step t+1 at row yr - 1
      if (j >= 4) {
        inner(S0, S1, S2, K0, yr - 2, 1, U2);             // step t+2 at row yr - 2
        if (j >= 6) {
          // step t+3 at row yr - 3 (one of the strip's rows)
          const int y3 = yr - 3;
          T g[9];
          pair_pull(U0, U1, U2, g);
          const uint32_t o3 = uint32_t(y3) * uint32_t(L.pitch) * uint32_t(sizeof(S)) + w.off;
          T fx3 = T(0), fy3 = T(0), dm3 = T(0);
          if (out_col && pair_node<T, MRT>(L, KM, y3, U1, g, true, fx3, fy3, dm3)) {
            if constexpr (HOLD) {
#pragma unroll
              for (int q = 0; q < 9; ++q) H[q] = g[q];
              oh = o3;
              held = true;
            } else {
#pragma unroll
              for (int q = 0; q < 9; ++q)
                Store<S>::st_cached(
                    reinterpret_cast<S*>(reinterpret_cast<char*>(B + int64_t(q) * L.plane) + o3), g[q]);
            }
          }
          fx[2] += double(fx3);
          fy[2] += double(fy3);
          dm[2] += double(dm3);
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          U0[q] = U1[q];
          U1[q] = U2[q];
        }
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        S0[q] = S1[q];
        S1[q] = S2[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      R0[q] = R1[q];
      R1[q] = R2[q];
    }
    KM = K0;
    K0 = K1;
    K1 = K2;
  }
  if constexpr (HOLD) flush();
  // one slot per wave and step: [k n, (k + 1) n) for step k
  const int n = L.tri_nslots;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = wave_sum(fx[k]), b = wave_sum(fy[k]), c = wave_sum(dm[k]);
    if (w.lane == 0) {
      double* o = part + int64_t(kPartials) * (int64_t(k) * n + slot);
      o[0] = a; o[1] = b; o[2] = c; o[3] = 0.0;
    }
  }
}

// ---- three steps per launch at the neural outlet (Sec. 3.1, Eq. 16) -----------
// An outlet block takes the three steps of the last kOutCols columns (nx-4 ..
// nx-1) for kOutRows3 rows y0 .. y0+55; the strips stop at column nx-5 and
// never read what the block computes (their cone stays three columns short
// of the outlet).  The block stages A_t over columns nx-7 .. nx-1 and rows
// y0-3 .. y0+58, takes step t+1 on columns nx-6 .. nx-1 for rows y0-2 ..
// y0+57, step t+2 on columns nx-5 .. nx-1 for rows y0-1 .. y0+56, and step
// t+3 on its own columns and rows; the outlet column of each step through
// the network (one 64-row tile per step, the rows past a step's own unused).
// 56 rows keep the block's LDS under 40 KB: the strips of the same launch
// reserve it too, and four workgroups per CU is what their registers allow.
// The strip-height rule counts the blocks' waves (tri_rows): at 4096 x 1024
// the 18-row strips and the 19 blocks overfilled four waves per SIMD, seven
// strip workgroups waited for a second round, and a launch took 118.1 us
// (134.7k MLUPS with 19-row strips, 0.96 of the Zou & He step).  Every node runs the single-step
// node code and the states between the steps are rounded as a store would
// round them, so the result is that of three single steps.  Force, mass and
// fallbacks of each step are counted on the block's own rows and columns.
template <typename S>
using T_of = typename Store<S>::T;
constexpr int kOutRows3 = kNnRows - 8;      // rows per three-step outlet block
constexpr int kSt3Rows = kOutRows3 + 6;     // staged rows y0-3 .. y0+58
constexpr int kSt3Cols = kOutCols + 3;      // staged columns nx-7 .. nx-1
constexpr int kT1Rows = kOutRows3 + 4;      // step t+1 rows y0-2 .. y0+57
constexpr int kT1Cols = kOutCols + 2;       // step t+1 columns nx-6 .. nx-1
constexpr int kT2Rows = kOutRows3 + 2;      // step t+2 rows y0-1 .. y0+56
constexpr int kT2Cols = kOutCols + 1;       // step t+2 columns nx-5 .. nx-1
static_assert(kT1Rows <= kNnRows, "one network tile per step");

template <typename T>
struct alignas(16) Nn3Smem {
  // A_t is dead once step t+1 has pulled it; the post-collision state of
  // step t+2 and the network activations (live together) then take its
  // memory, side by side
  union {
    T st[9 * kSt3Rows * kSt3Cols];
    struct {
      T t2[9 * kT2Rows * kT2Cols];
      MlpH H;
    } late;
  } u;
  T t1[9 * kT1Rows * kT1Cols];       // post-collision state of step t+1
  MlpX X;
  T prev[kNnRows * 4];               // g3, g6, g7, density offset at x = L-1
};
static_assert(sizeof(Nn3Smem<float>) <= 40 * 1024, "four workgroups per CU");

// One intermediate step of an outlet block: the interior column c (of the
// source tile src[R][C], whose last column is the outlet) for block row j
// (tile row j + 1 of src), result into dst[q][j][c - 1]; features of the
// columns L-1 .. L-3 and prev at L-1 for the network.  `own`: count force and
// mass (the block's own rows and columns).
template <typename S, int MRT, int R, int C, int DR, int DC>
__device__ __forceinline__ void nn3_interior(const StepLaunch& L, const MlpDev* w, const T_of<S>* src,
                                             T_of<S>* dst, MlpX& X, T_of<S>* prev, int j, int c,
                                             uint32_t lk, bool own, double& fx, double& fy, double& dm) {
  using T = T_of<S>;
  T g[9];
  tile_pull<T, R, C>(src, j + 1, c, lk, g);
  const bool live = !(lk & LINK_SOLID);
  const int jc = C - 2 - c;                   // column x = L-1-jc
  if (jc >= 0 && jc <= 2) {
#pragma unroll
    for (int q = 0; q < 9; ++q)
      X.x[j * kXPitch + 9 * jc + q] = live ? feature_bf16(w, 9 * jc + q, float(g[q])) : 0;
    if (jc == 0) {
      prev[j * 4 + 0] = g[3];
      prev[j * 4 + 1] = g[6];
      prev[j * 4 + 2] = g[7];
      prev[j * 4 + 3] = macro(g).drho;
    }
  }
  if (live) {
    if (own) {
      T fxk = T(0), fyk = T(0);
      add_force(lk, g, fxk, fyk);
      fx += double(fxk);
      fy += double(fyk);
      dm += double(macro(g).drho);
    }
    collide<T, MRT>(g, L);
  } else {
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = src[(q * R + j + 1) * C + c];
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) dst[(q * DR + j) * DC + c - 1] = Store<S>::stored(g[q]);
}

// The outlet node of block row j of an intermediate step: the pull of its
// known populations from src (whose last column is the outlet).
template <typename T, int R, int C>
__device__ __forceinline__ void nn3_outlet_pull(const T* src, int j, uint32_t lko, T go[9]) {
  tile_pull<T, R, C>(src, j + 1, C - 1, lko, go);
  if (lko & LINK_SOLID) {
#pragma unroll
    for (int q = 0; q < 9; ++q) go[q] = src[(q * R + j + 1) * C + C - 1];
  }
}

template <typename S, int MRT>
__device__ void nn3_block(const StepLaunch& L, int nb, Nn3Smem<T_of<S>>& sm, double* part, int slot) {
  using T = T_of<S>;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const MlpDev* __restrict__ w = L.mlp;
  const int y0 = nb * kOutRows3;
  const int xs0 = L.nx - kSt3Cols;           // first staged column
  const int tid = threadIdx.x;
  const int j = tid & 63, k = tid >> 6;
  double fx[3] = {0, 0, 0}, fy[3] = {0, 0, 0}, dm[3] = {0, 0, 0}, nf[3] = {0, 0, 0};

  // the link words of this thread's nodes in the three steps, loaded with
  // the stage below (the block's chain of steps is its latency): step t+1
  // rows y0-2+j, columns nx-7+c for c = 5-k (and c = 1, k = 0); step t+2
  // rows y0-1+j, column nx-6+(4-k); the outlet column (k = 0); step t+3 row
  // y0+j, column nx-4+k
  auto link_at = [&](int yrel, int x) -> uint32_t {
    const int yb = block_row(L, y0 + yrel);
    return yb >= 0 ? L.links[int64_t(yb) * L.pitch + x] : LINK_SOLID;
  };
  uint32_t lk1[2] = {LINK_SOLID, LINK_SOLID}, lk2[2] = {LINK_SOLID, LINK_SOLID};
  uint32_t lko[2] = {LINK_SOLID, LINK_SOLID};
  if (j < kT1Rows) {
    lk1[0] = link_at(j - 2, L.nx - 7 + (5 - k));
    if (k == 0) {
      lk1[1] = link_at(j - 2, L.nx - 7 + 1);
      lko[0] = link_at(j - 2, L.nx - 1);
    }
  }
  if (j < kT2Rows) {
    lk2[0] = link_at(j - 1, L.nx - 6 + (4 - k));
    if (k == 0) lko[1] = link_at(j - 1, L.nx - 1);
  }
  const bool row_ok = j < kOutRows3 && y0 + j < L.ny;
  const uint32_t lk3 = row_ok ? L.links[int64_t(y0 + j) * L.pitch + L.nx - 4 + k] : LINK_SOLID;

  // 1. stage A_t[q][y0-3 .. y0+58][nx-7 .. nx-1], every load of a thread
  // issued before the first is waited for
  constexpr int kStN = 9 * kSt3Rows * kSt3Cols;
#pragma unroll
  for (int it = 0; it < (kStN + kBlock - 1) / kBlock; ++it) {
    const int i = tid + it * kBlock;
    if (i < kStN) {
      const int q = i / (kSt3Rows * kSt3Cols);
      const int rem = i - q * (kSt3Rows * kSt3Cols);
      const int r = rem / kSt3Cols, c = rem - r * kSt3Cols;
      int y = y0 - 3 + r;
      y = L.yper ? (y + 3 * L.ny) % L.ny : min(max(y, 0), L.ny - 1);   // clamped rows: never pulled
      sm.u.st[i] = Store<S>::ld(A + int64_t(q) * L.plane + int64_t(y) * L.pitch + xs0 + c);
    }
  }
  __syncthreads();

  // One intermediate step (step index h) from tile src (R x C, outlet last)
  // into dst (DR x DC): interior columns 1 .. C-2 of src, then the outlet
  // through the network.  Block rows j = 0 .. DR-1 are rows y0 - (2 - h) + j.
  auto step = [&](auto src, auto dst, auto Rc, auto Cc, auto DRc, auto DCc, int h,
                  const uint32_t* lki, uint32_t lkout) {
    constexpr int R = decltype(Rc)::value, C = decltype(Cc)::value;
    constexpr int DR = decltype(DRc)::value, DC = decltype(DCc)::value;
    const int yrel = j - (2 - h);                        // row relative to y0
    const bool row_in = j < DR;
    const bool own_row = row_in && yrel >= 0 && yrel < kOutRows3 && y0 + yrel < L.ny;
    // interior columns 1 .. C-2: thread k takes columns C-2-k, C-6-k, ...
    int it = 0;
    for (int c = (C - 2) - k; c >= 1; c -= 4, ++it) {
      if (row_in) {
        const bool own = own_row && c >= C - kOutCols;  // own columns nx-4 .. nx-2
        nn3_interior<S, MRT, R, C, DR, DC>(L, w, src, dst, sm.X, sm.prev, j, c, lki[it], own,
                                           fx[h], fy[h], dm[h]);
      } else if (c >= C - 4) {
        // rows past the step's own rows: no features for the tile
        const int jc = C - 2 - c;
#pragma unroll
        for (int q = 0; q < 9; ++q) sm.X.x[j * kXPitch + 9 * jc + q] = 0;
      }
    }
    if (k == 0) {
#pragma unroll
      for (int f = 27; f < 32; ++f) sm.X.x[j * kXPitch + f] = 0;
    }
    T go[9];
    if (k == 0 && row_in) nn3_outlet_pull<T, R, C>(src, j, lkout, go);
    __syncthreads();                      // features, prev
    mlp_tile(w, sm.X, sm.u.late.H);
    if (k == 0 && row_in) {
      if (!(lkout & LINK_SOLID)) {
        T fxk = T(0), fyk = T(0);
        if (own_row) add_force(lkout, go, fxk, fyk);
        const bool kept = nn_reconstruct(w, &sm.u.late.H.o[j * 4], &sm.prev[j * 4], go,
                                         T(L.one_minus_rho_out));
        if (own_row) {
          fx[h] += double(fxk);
          fy[h] += double(fyk);
          dm[h] += double(macro(go).drho);
          nf[h] += kept ? 0.0 : 1.0;
        }
        collide<T, MRT>(go, L);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) dst[(q * DR + j) * DC + DC - 1] = Store<S>::stored(go[q]);
    }
    __syncthreads();                      // dst complete; H read
  };
  step(sm.u.st, sm.t1, std::integral_constant<int, kSt3Rows>{}, std::integral_constant<int, kSt3Cols>{},
       std::integral_constant<int, kT1Rows>{}, std::integral_constant<int, kT1Cols>{}, 0, lk1,
       lko[0]);
  step(sm.t1, sm.u.late.t2, std::integral_constant<int, kT1Rows>{}, std::integral_constant<int, kT1Cols>{},
       std::integral_constant<int, kT2Rows>{}, std::integral_constant<int, kT2Cols>{}, 1, lk2,
       lko[1]);

  // 3. step t+3 on the block's own rows y0 + j (j < 56): columns nx-4 .. nx-2
  // (k = 0 .. 2), the outlet column (k = 3)
  const int y = y0 + j;
  const uint32_t lk = lk3;
  T g[9];
  // rows j >= kOutRows3 are no output rows: their (unused) pull stays inside t2
  tile_pull<T, kT2Rows, kT2Cols>(sm.u.late.t2, min(j, kOutRows3 - 1) + 1, k + 1, lk, g);
  const bool live = row_ok && !(lk & LINK_SOLID);
  if (k < 3) {
    const int jc = 2 - k;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      sm.X.x[j * kXPitch + 9 * jc + q] = live ? feature_bf16(w, 9 * jc + q, float(g[q])) : 0;
    if (k == 2) {
      sm.prev[j * 4 + 0] = g[3];
      sm.prev[j * 4 + 1] = g[6];
      sm.prev[j * 4 + 2] = g[7];
      sm.prev[j * 4 + 3] = macro(g).drho;
    }
    if (live) {
      T fxk = T(0), fyk = T(0);
      add_force(lk, g, fxk, fyk);
      fx[2] += double(fxk);
      fy[2] += double(fyk);
      dm[2] += double(macro(g).drho);
      collide<T, MRT>(g, L);
      const int64_t row = int64_t(y) * L.pitch + L.nx - 4 + k;
#pragma unroll
      for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row, g[q]);
    }
  } else {
#pragma unroll
    for (int f = 27; f < 32; ++f) sm.X.x[j * kXPitch + f] = 0;
  }
  __syncthreads();
  mlp_tile(w, sm.X, sm.u.late.H);
  if (k == 3 && live) {
    T fxk = T(0), fyk = T(0);
    add_force(lk, g, fxk, fyk);
    const bool kept = nn_reconstruct(w, &sm.u.late.H.o[j * 4], &sm.prev[j * 4], g,
                                     T(L.one_minus_rho_out));
    fx[2] += double(fxk);
    fy[2] += double(fyk);
    dm[2] += double(macro(g).drho);
    nf[2] += kept ? 0.0 : 1.0;
    collide<T, MRT>(g, L);
    const int64_t row = int64_t(y) * L.pitch + L.nx - 1;
#pragma unroll
    for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row, g[q]);
  }
  // one slot per wave and step, as the strips
  const int n = L.tri_nslots;
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    const double a = wave_sum(fx[h]), b = wave_sum(fy[h]), c = wave_sum(dm[h]), d = wave_sum(nf[h]);
    if (j == 0) {
      double* o = part + int64_t(kPartials) * (int64_t(h) * n + slot + k);
      o[0] = a; o[1] = b; o[2] = c; o[3] = d;
    }
  }
}

// ---- three steps per launch at the characteristic outlet (Sec. 4) --------------
// The geometry of the three-step neural blocks with kCbRows3 own rows: A_t
// staged over columns nx-7 .. nx-1 and rows y0-3 .. y0+50 (rows wrapped:
// periodic laterals), step t+1 on columns nx-6 .. nx-1 for rows y0-2 ..
// y0+49, step t+2 on columns nx-5 .. nx-1 for rows y0-1 .. y0+48, step t+3
// on the own columns and rows.  The outlet column of each step takes the
// LODI update of the moments of the state before it (columns nx-3 .. nx-1),
// the tuning network's features taking the time derivatives of the step
// before: from L.cbc_dt for step t+1, from LDS for the next two; step t+3's
// derivatives of the own rows go to L.cbc_dt_w.  48 rows keep the block's
// LDS under 40 KB (four workgroups per CU, as for the strips).
constexpr int kCbRows3 = 48;
constexpr int kCSt3Rows = kCbRows3 + 6;     // staged rows y0-3 .. y0+50
constexpr int kCT1Rows = kCbRows3 + 4;      // step t+1 rows y0-2 .. y0+49
constexpr int kCT2Rows = kCbRows3 + 2;      // step t+2 rows y0-1 .. y0+48
static_assert(kCT1Rows <= kNnRows, "one network tile per step");

template <typename T>
struct alignas(16) Cbc3Smem {
  union {
    T st[9 * kCSt3Rows * kSt3Cols];  // A_t (dead once step t+1 is done)
    T t2[9 * kCT2Rows * kT2Cols];    // post-collision state of step t+2
  } u;
  T t1[9 * kCT1Rows * kT1Cols];      // post-collision state of step t+1
  T mo[3 * 3 * kCSt3Rows];           // moments of the last three columns of the state in use
  T dt[2][kNnRows * 3];              // p_t, u_t, v_t of steps t+1 and t+2 per block row
  CbcNetSmem<T> net;
};
static_assert(sizeof(Cbc3Smem<float>) <= 40 * 1024, "four workgroups per CU");

template <typename S, int MRT>
__device__ void cbc3_block(const StepLaunch& L, int nb, Cbc3Smem<T_of<S>>& sm, double* part, int slot) {
  using T = T_of<S>;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const CbcDev* __restrict__ c = L.cbc;
  const int y0 = nb * kCbRows3;
  const int xs0 = L.nx - kSt3Cols;
  const int tid = threadIdx.x;
  const int j = tid & 63, k = tid >> 6;
  double fx[3] = {0, 0, 0}, fy[3] = {0, 0, 0}, dm[3] = {0, 0, 0};

  // 1. stage A_t[q][y0-3 .. y0+50][nx-7 .. nx-1] (rows wrapped)
  constexpr int kStN = 9 * kCSt3Rows * kSt3Cols;
#pragma unroll
  for (int it = 0; it < (kStN + kBlock - 1) / kBlock; ++it) {
    const int i = tid + it * kBlock;
    if (i < kStN) {
      const int q = i / (kCSt3Rows * kSt3Cols);
      const int rem = i - q * (kCSt3Rows * kSt3Cols);
      const int r = rem / kSt3Cols, cc = rem - r * kSt3Cols;
      const int y = (y0 - 3 + r + 3 * L.ny) % L.ny;
      sm.u.st[i] = Store<S>::ld(A + int64_t(q) * L.plane + int64_t(y) * L.pitch + xs0 + cc);
    }
  }
  __syncthreads();

  // One intermediate step (index h) from tile src (R x C, outlet last) into
  // dst (DR x DC): block rows j = 0 .. DR-1 are rows y0 - (2 - h) + j; the
  // moments of src's last three columns are taken first; the outlet's
  // previous time derivatives come from prevdt (NULL: L.cbc_dt), its new
  // ones go to sm.dt[h].
  auto step = [&](const T* src, T* dst, auto Rc, auto Cc, auto DRc, auto DCc, int h) {
    constexpr int R = decltype(Rc)::value, C = decltype(Cc)::value;
    constexpr int DR = decltype(DRc)::value, DC = decltype(DCc)::value;
    tile_moments<T, R, C>(src, C - 3, sm.mo);
    const int yrel = j - (2 - h);
    const bool row_in = j < DR;
    const int yb = (y0 + yrel + 2 * L.ny) % L.ny;
    const bool own_row = row_in && yrel >= 0 && yrel < kCbRows3 && y0 + yrel < L.ny;
    // interior columns 1 .. C-2: thread k takes columns C-2-k, C-6-k, ...
    for (int cc = (C - 2) - k; cc >= 1; cc -= 4) {
      if (!row_in) continue;
      const int x = L.nx - C + cc;
      const uint32_t lk = L.links[int64_t(yb) * L.pitch + x];
      const bool own = own_row && cc >= C - kOutCols;
      T g[9];
      tile_pull<T, R, C>(src, j + 1, cc, lk, g);
      if (!(lk & LINK_SOLID)) {
        if (own) {
          T fxk = T(0), fyk = T(0);
          add_force(lk, g, fxk, fyk);
          fx[h] += double(fxk);
          fy[h] += double(fyk);
          dm[h] += double(macro(g).drho);
        }
        collide<T, MRT>(g, L);
      } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = src[(q * R + j + 1) * C + cc];
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) dst[(q * DR + j) * DC + cc - 1] = Store<S>::stored(g[q]);
    }
    __syncthreads();                      // moments of src
    T sigma = T(c->sigma), kappa2 = T(c->kappa2);
    if (c->has_net) {
      if (tid < kNnRows) {
        const int r = min(j, DR - 1) + 1;   // rows past the step's own: unused
        T g6[6];
        cbc_gradients<T, R>(sm.mo, r, g6);
        T prev[3];
        if (h == 0) {
          const double* d = L.cbc_dt + 4 * int64_t((y0 + min(j, DR - 1) - 2 + 2 * L.ny) % L.ny);
          prev[0] = T(d[0]); prev[1] = T(d[1]); prev[2] = T(d[2]);
        } else {
          // the previous step's rows are shifted by one against this step's
          const int rp = min(j, DR - 1) + 1;
          prev[0] = sm.dt[h - 1][rp * 3 + 0];
          prev[1] = sm.dt[h - 1][rp * 3 + 1];
          prev[2] = sm.dt[h - 1][rp * 3 + 2];
        }
        cbc_features(c, g6, prev, &sm.net.feat[j * kCbcIn]);
      }
      cbc_network(c, sm.net, sigma, kappa2);
    }
    if (tid < kNnRows && row_in) {
      const uint32_t lk = L.links[int64_t(yb) * L.pitch + L.nx - 1];
      T g[9];
      tile_pull<T, R, C>(src, j + 1, C - 1, lk, g);
      if (!(lk & LINK_SOLID)) {
        const int r = j + 1;
        T g6[6], nst[3], dtn[3];
        cbc_gradients<T, R>(sm.mo, r, g6);
        cbc_lodi(c, g6, sm.mo[(0 * 3 + 2) * R + r], sm.mo[(1 * 3 + 2) * R + r],
                 sm.mo[(2 * 3 + 2) * R + r], sigma, kappa2, nst, dtn);
        sm.dt[h][j * 3 + 0] = dtn[0];
        sm.dt[h][j * 3 + 1] = dtn[1];
        sm.dt[h][j * 3 + 2] = dtn[2];
        outlet_state(g, nst[0], nst[1], nst[2]);
        if (own_row) {
          T fxk = T(0), fyk = T(0);
          add_force(lk, g, fxk, fyk);
          fx[h] += double(fxk);
          fy[h] += double(fyk);
          dm[h] += double(macro(g).drho);
        }
        collide<T, MRT>(g, L);
      } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = src[(q * R + j + 1) * C + C - 1];
        sm.dt[h][j * 3 + 0] = sm.dt[h][j * 3 + 1] = sm.dt[h][j * 3 + 2] = T(0);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) dst[(q * DR + j) * DC + DC - 1] = Store<S>::stored(g[q]);
    }
    __syncthreads();                      // dst complete; the moments and src read
  };
  step(sm.u.st, sm.t1, std::integral_constant<int, kCSt3Rows>{}, std::integral_constant<int, kSt3Cols>{},
       std::integral_constant<int, kCT1Rows>{}, std::integral_constant<int, kT1Cols>{}, 0);
  step(sm.t1, sm.u.t2, std::integral_constant<int, kCT1Rows>{}, std::integral_constant<int, kT1Cols>{},
       std::integral_constant<int, kCT2Rows>{}, std::integral_constant<int, kT2Cols>{}, 1);

  // 3. step t+3 on the own rows y0 + j (j < 48): columns nx-4 .. nx-2 (k < 3)
  tile_moments<T, kCT2Rows, kT2Cols>(sm.u.t2, kT2Cols - 3, sm.mo);
  const int y = y0 + j;
  const bool row_ok = j < kCbRows3 && y < L.ny;
  if (k < 3 && row_ok) {
    const uint32_t lk = L.links[int64_t(y) * L.pitch + L.nx - 4 + k];
    if (!(lk & LINK_SOLID)) {
      T g[9];
      tile_pull<T, kCT2Rows, kT2Cols>(sm.u.t2, j + 1, k + 1, lk, g);
      T fxk = T(0), fyk = T(0);
      add_force(lk, g, fxk, fyk);
      fx[2] += double(fxk);
      fy[2] += double(fyk);
      dm[2] += double(macro(g).drho);
      collide<T, MRT>(g, L);
      const int64_t off = int64_t(y) * L.pitch + L.nx - 4 + k;
#pragma unroll
      for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + off, g[q]);
    }
  }
  __syncthreads();                      // moments of step t+2
  T sigma = T(c->sigma), kappa2 = T(c->kappa2);
  if (c->has_net) {
    if (tid < kNnRows) {
      const int r = min(j, kCbRows3 - 1) + 1;    // rows j >= 48: unused
      T g6[6];
      cbc_gradients<T, kCT2Rows>(sm.mo, r, g6);
      const T prev[3] = {sm.dt[1][r * 3 + 0], sm.dt[1][r * 3 + 1], sm.dt[1][r * 3 + 2]};
      cbc_features(c, g6, prev, &sm.net.feat[j * kCbcIn]);
    }
    cbc_network(c, sm.net, sigma, kappa2);
  }
  if (tid < kNnRows && row_ok) {
    const uint32_t lk = L.links[int64_t(y) * L.pitch + L.nx - 1];
    if (!(lk & LINK_SOLID)) {
      const int r = j + 1;
      T g[9], g6[6], nst[3], dtn[3];
      tile_pull<T, kCT2Rows, kT2Cols>(sm.u.t2, r, kT2Cols - 1, lk, g);
      cbc_gradients<T, kCT2Rows>(sm.mo, r, g6);
      cbc_lodi(c, g6, sm.mo[(0 * 3 + 2) * kCT2Rows + r], sm.mo[(1 * 3 + 2) * kCT2Rows + r],
               sm.mo[(2 * 3 + 2) * kCT2Rows + r], sigma, kappa2, nst, dtn);
      double* d = L.cbc_dt_w + 4 * int64_t(y);
      d[0] = double(dtn[0]);
      d[1] = double(dtn[1]);
      d[2] = double(dtn[2]);
      outlet_state(g, nst[0], nst[1], nst[2]);
      T fxk = T(0), fyk = T(0);
      add_force(lk, g, fxk, fyk);
      fx[2] += double(fxk);
      fy[2] += double(fyk);
      dm[2] += double(macro(g).drho);
      collide<T, MRT>(g, L);
      const int64_t off = int64_t(y) * L.pitch + L.nx - 1;
#pragma unroll
      for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + off, g[q]);
    } else {
      double* d = L.cbc_dt_w + 4 * int64_t(y);
      d[0] = d[1] = d[2] = 0.0;
    }
  }
  const int n = L.tri_nslots;
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    const double a = wave_sum(fx[h]), b = wave_sum(fy[h]), cc = wave_sum(dm[h]);
    if (j == 0) {
      double* o = part + int64_t(kPartials) * (int64_t(h) * n + slot + k);
      o[0] = a; o[1] = b; o[2] = cc; o[3] = 0.0;
    }
  }
}

constexpr int kTriSpecial = (1 + 3 * kReducers + 7) / 8 * 8;

// OUT: 0 the Zou & He outlet inside the strips; OUTLET_NN the neural outlet
// blocks (the first tri_out workgroups after the reducers).
template <typename S, int MRT, int OUT, int HOLD>
__global__ void __launch_bounds__(kBlock) k_step3(const StepLaunch L) {
  const int v = int(blockIdx.x);
  if (v < kTriSpecial) {
    if (v == 0) {
      if (L.reduce2) multi_level2<3>(L.lvl_r, L);
    } else if (v <= 3 * kReducers && L.reduce1) {
      multi_level1(static_cast<const double*>(L.part_r), v - 1, L.tri_nslots, L);
    }
    return;
  }
  const int b = v - kTriSpecial;
  double* part = static_cast<double*>(L.part_w);
  if constexpr (OUT == OUTLET_NN) {
    if (b < L.tri_out) {
      __shared__ Nn3Smem<T_of<S>> sm;
      nn3_block<S, MRT>(L, b, sm, part, b * kWaves);
      return;
    }
  } else if constexpr (OUT == OUTLET_CBC) {
    if (b < L.tri_out) {
      __shared__ Cbc3Smem<T_of<S>> sm;
      cbc3_block<S, MRT>(L, b, sm, part, b * kWaves);
      return;
    }
  }
  int sb = b - L.tri_out;
  const int nsb = int(gridDim.x) - kTriSpecial - L.tri_out;
  sb = L.tri_chunk > 0 ? xcd_remap_chunks(sb, nsb, L.tri_chunk) : xcd_remap(sb, nsb);
  const int slot = __builtin_amdgcn_readfirstlane((L.tri_out + sb) * kWaves + int(threadIdx.x >> 6));
  if (slot >= L.tri_nslots) return;                  // whole wave
  tri_strip<S, MRT, HOLD>(L, slot - L.tri_out * kWaves, slot, part);
}

template <typename S, int MRT, int HOLD>
static hipError_t launch_tri_h(const StepLaunch& L, hipStream_t s) {
  const int blocks = kTriSpecial + (L.tri_nslots + kWaves - 1) / kWaves;
  if (L.tri_out > 0 && L.outlet == OUTLET_NN)
    hipLaunchKernelGGL((k_step3<S, MRT, OUTLET_NN, HOLD>), dim3(blocks), dim3(kBlock), 0, s, L);
  else if (L.tri_out > 0 && L.outlet == OUTLET_CBC)
    hipLaunchKernelGGL((k_step3<S, MRT, OUTLET_CBC, HOLD>), dim3(blocks), dim3(kBlock), 0, s, L);
  else if (L.tri_out == 0)
    hipLaunchKernelGGL((k_step3<S, MRT, 0, HOLD>), dim3(blocks), dim3(kBlock), 0, s, L);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename S, int MRT>
static hipError_t launch_tri_t(const StepLaunch& L, hipStream_t s) {
  if constexpr (!std::is_same_v<S, __half>) {
    if (L.tri_hold) return launch_tri_h<S, MRT, 1>(L, s);
  }
  return L.tri_hold ? hipErrorInvalidValue : launch_tri_h<S, MRT, 0>(L, s);
}

int tri_waves(int nx, int ny, int rows) {
  return ((nx + kTriCols - 1) / kTriCols) * ((ny + rows - 1) / rows);
}

int strip_rows(int nx, int ny, int pitch_bytes, int cols, int reserved_waves, int max_rows);   // below

int tri_rows(int nx, int ny, int pitch_bytes, int outlet_blocks) {
  return strip_rows(nx, ny, pitch_bytes, kTriCols, outlet_blocks * kWaves, kTriRowsMax);
}

int tri_chunk(int tri_nx) { return ((tri_nx + kTriCols - 1) / kTriCols + kWaves - 1) / kWaves; }

int tri_outlet_blocks(int ny, bool cbc) {
  const int rows = cbc ? kCbRows3 : kOutRows3;
  return (ny + rows - 1) / rows;
}

// FP32 and FP16 offsets (the FP64 variant would need twice the registers).
bool tri_supported(int precision) { return precision != LBM_FP64; }

hipError_t launch_triple(const StepLaunch& L, hipStream_t s) {
  switch (L.precision * 2 + L.collision) {
    case LBM_FP32_OFFSET * 2 + LBM_BGK: return launch_tri_t<float, 0>(L, s);
    case LBM_FP32_OFFSET * 2 + LBM_MRT: return launch_tri_t<float, 1>(L, s);
    case LBM_FP16_OFFSET * 2 + LBM_BGK: return launch_tri_t<__half, 0>(L, s);
    case LBM_FP16_OFFSET * 2 + LBM_MRT: return launch_tri_t<__half, 1>(L, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_finalize_triple(const StepLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((k_finalize_multi<double, 3>), dim3(1), dim3(kBlock), 0, s, L, L.tri_nslots);
  return hipGetLastError();
}

// Whether the strips hold their step-(t+2) stores back by one row (with
// the link flags of the whole strip read first).  The plain walk waits for
// the next row's loads (and the stores before them) as soon as it has
// issued them; the held walk waits for them only after the row's work.
// That pays where the populations come from HBM, and loses where much of
// both buffers stays in the 256 MB last-level cache.  Measured (MRT, MLUPS,
// plain / held): FP32 4096 x 1024 (151 MB per buffer) 111.5k / 102.0k,
// 6144 x 512 131.6k / 119.4k, 3072 x 1024 131.6k / 119.8k, 4096 x 1536
// (226 MB) 88.9k / 102.0k, 4096 x 2048 99.6k / 105.5k, 8192 x 2048
// 106.6k / 109.6k, 8192 x 4096 110.3k / 115.0k, 16384 x 4096 114.0k /
// 120.9k; FP64 16384 x 4096 60.3k / 66.0k, 4096 x 1024 (302 MB) 52.2k /
// 51.9k; FP16 16384 x 4096 186.0k / 146.1k (never held).
int pair_hold(int precision, int64_t buffer_bytes) {
  return precision != LBM_FP16_OFFSET && buffer_bytes > int64_t(200) * 1000 * 1000;
}

int pair_waves(int nx, int ny, int rows) {
  return ((nx + kPairCols - 1) / kPairCols) * ((ny + rows - 1) / rows);
}

// Output rows per strip.  The shortest strips (least halo per wave is the
// longest) that keep the grid within four waves per SIMD (4096 waves: all
// resident at once with room to spare; outlet blocks of the same launch,
// reserved_waves, count against them, since they last as long as a strip),
// between 12 and max_rows rows (18 for two steps per launch, 24 for three:
// with the neural outlet's 76 waves the 4096 x 1024 grid needs 19); a height
// above 12 whose band stride (rows x row bytes) is a multiple of 64 KiB is
// moved by one row, since bands that start on such strides met the same
// HBM channels (4096 x 1024 FP32: 16 rows 104.9k, 18 rows 111.7k MLUPS).
// Measured against fixed heights (MLUPS, FP32): 4096 x 1024 18 rows 111.7k
// (24: 102.2k, best of 12-24); 4096 x 512 12 rows 114.1k (24: 79.7k);
// 6144 x 512 14 rows 131.3k (24: 106.1k); 3072 x 1024 14 rows 131.8k;
// 2048 x 2048 18 rows 108.8k; 8192 x 2048 17 rows 106.7k (12: 109.2k);
// 16384 x 4096 17 rows 114.0k (16: 115.0k, 24: 110.6k); FP16 4096 x 1024
// 143.7k (24: 127.6k); FP64 4096 x 1024 52.2k (24: 53.2k).
constexpr int kSimds = 256 * 4;      // the MI355X's 256 CUs of four SIMDs each
int strip_rows(int nx, int ny, int pitch_bytes, int cols, int reserved_waves, int max_rows) {
  const int strips = (nx + cols - 1) / cols;
  const int bands = std::max(1, (4 * kSimds - reserved_waves) / strips);
  int rows = std::min(std::max((ny + bands - 1) / bands, kPairRowsMin), max_rows);
  if (rows > kPairRowsMin && (int64_t(rows) * pitch_bytes) % 65536 == 0)
    rows += rows < max_rows ? 1 : -1;
  return rows;
}

int pair_rows(int nx, int ny, int pitch_bytes) {
  return strip_rows(nx, ny, pitch_bytes, kPairCols, 0, kPairRowsMax);
}

int pair_outlet_blocks(int ny) { return (ny + kOutRows - 1) / kOutRows; }

// Strip workgroups are dealt to the XCDs in chunks of one band (the
// workgroups of one row of strips), XCD x taking chunks x, x + 8, ...: the
// lines that x-adjacent strips share then meet in one L2.  Against dispatch
// order (MLUPS, FP32): 4096 x 1024 99.0k -> 102.4k, 4096 x 2048 84.8k ->
// 89.3k, 8192 x 2048 97.7k -> 104.5k, 16384 x 4096 107.6k -> 110.8k; FP16 and
// FP64 at 4096 x 1024 +1 %.  Chunks of two or four bands and one contiguous
// eighth per XCD were within 2 % of it (eighths 1 % ahead at 16384 x 4096
// and 3 % in FP64, 1-2 % behind elsewhere).
int pair_chunk(int pair_nx) {
  return ((pair_nx + kPairCols - 1) / kPairCols + kWaves - 1) / kWaves;
}

int pair_outlet_cols() { return kOutCols; }

hipError_t launch_pair(const StepLaunch& L, hipStream_t s) {
  switch (L.precision * 2 + L.collision) {
    case LBM_FP64 * 2 + LBM_BGK: return launch_pair_t<double, 0>(L, s);
    case LBM_FP64 * 2 + LBM_MRT: return launch_pair_t<double, 1>(L, s);
    case LBM_FP32_OFFSET * 2 + LBM_BGK: return launch_pair_t<float, 0>(L, s);
    case LBM_FP32_OFFSET * 2 + LBM_MRT: return launch_pair_t<float, 1>(L, s);
    case LBM_FP16_OFFSET * 2 + LBM_BGK: return launch_pair_t<__half, 0>(L, s);
    case LBM_FP16_OFFSET * 2 + LBM_MRT: return launch_pair_t<__half, 1>(L, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_finalize_pair(const StepLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((k_finalize_multi<double, 2>), dim3(1), dim3(kBlock), 0, s, L,
                     L.pair_nslots);   // FP64 slots
  return hipGetLastError();
}

// ---- initialisation (Eq. 3 at rest density, noisy inlet velocity) -------------------
template <typename S>
__global__ void __launch_bounds__(kBlock) k_init(const InitLaunch L) {
  using T = typename Store<S>::T;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= int64_t(L.rows) * L.nx) return;
  const int r = int(i / L.nx), x = int(i - int64_t(r) * L.nx);
  const int y = L.y0 + r;
  const int64_t node = int64_t(y) * L.pitch + x;
  const bool solid = L.links[node] & LINK_SOLID;
  double rho = 1.0, ux = 0.0, uy = 0.0;
  if (!solid) {
    if (L.fields) {
      const int64_t n = int64_t(L.rows) * L.nx;
      rho = L.fields[i];
      ux = L.fields[n + i];
      uy = L.fields[2 * n + i];
    } else {
      const uint64_t k = 2ull * (uint64_t(y) * uint64_t(L.nx) + uint64_t(x)) + 1ull;
      ux = L.u_in + L.noise_amp * (2.0 * unit_double(splitmix64_at(L.seed, k)) - 1.0);
      uy = L.noise_amp * (2.0 * unit_double(splitmix64_at(L.seed, k + 1)) - 1.0);
    }
  }
  const double usq = 1.5 * (ux * ux + uy * uy);
  S* A = static_cast<S*>(L.A);
  S* B = static_cast<S*>(L.B);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double cu = cx(q) * ux + cy(q) * uy;
    const double geq = wgt<double>(q) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - usq));
    Store<S>::st_cached(A + int64_t(q) * L.plane + node, T(geq));
    Store<S>::st_cached(B + int64_t(q) * L.plane + node, T(geq));
  }
}

hipError_t launch_init(const InitLaunch& L, hipStream_t s) {
  const int64_t n = int64_t(L.rows) * L.nx;
  const dim3 grid(unsigned((n + kBlock - 1) / kBlock));
  switch (L.precision) {
    case LBM_FP64: hipLaunchKernelGGL(k_init<double>, grid, dim3(kBlock), 0, s, L); break;
    case LBM_FP32_OFFSET: hipLaunchKernelGGL(k_init<float>, grid, dim3(kBlock), 0, s, L); break;
    case LBM_FP16_OFFSET: hipLaunchKernelGGL(k_init<__half>, grid, dim3(kBlock), 0, s, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- read-out and write-back of the stored state ---------------------------------
template <typename S>
__global__ void __launch_bounds__(kBlock) k_read(const S* A, double* out, int nx, int pitch,
                                                 int64_t plane, int y0, int rows) {
  const int64_t n = int64_t(rows) * nx;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int r = int(i / nx), x = int(i - int64_t(r) * nx);
  const int64_t node = int64_t(y0 + r) * pitch + x;
#pragma unroll
  for (int q = 0; q < 9; ++q)
    out[q * n + i] = double(Store<S>::ld(A + q * plane + node)) + wgt<double>(q);
}

template <typename S>
__global__ void __launch_bounds__(kBlock) k_write(S* A, S* B, const double* in, int nx,
                                                  int pitch, int64_t plane, int y0, int rows) {
  using T = typename Store<S>::T;
  const int64_t n = int64_t(rows) * nx;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int r = int(i / nx), x = int(i - int64_t(r) * nx);
  const int64_t node = int64_t(y0 + r) * pitch + x;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const T v = T(in[q * n + i] - wgt<double>(q));
    Store<S>::st_cached(A + q * plane + node, v);
    Store<S>::st_cached(B + q * plane + node, v);
  }
}

// Moments of the stored state in FP64 (Eq. 4): rho = 1 + sum of the offsets,
// j = sum_i c_i g_i (the weights carry no momentum), u = j / rho.
template <typename S>
__global__ void __launch_bounds__(kBlock) k_macro(const S* A, double* out, int nx, int pitch,
                                                  int64_t plane, int y0, int rows) {
  const int64_t n = int64_t(rows) * nx;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int r = int(i / nx), x = int(i - int64_t(r) * nx);
  const int64_t node = int64_t(y0 + r) * pitch + x;
  double g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) g[q] = double(Store<S>::ld(A + q * plane + node));
  const Macro<double> m = macro(g);
  out[i] = m.rho;
  out[n + i] = m.jx / m.rho;
  out[2 * n + i] = m.jy / m.rho;
}

hipError_t launch_macro(int precision, const void* A, double* out, int nx, int pitch,
                        int64_t plane, int y0, int rows, hipStream_t s) {
  const dim3 grid(unsigned((int64_t(rows) * nx + kBlock - 1) / kBlock));
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(k_macro<double>, grid, dim3(kBlock), 0, s,
                         static_cast<const double*>(A), out, nx, pitch, plane, y0, rows);
      break;
    case LBM_FP32_OFFSET:
      hipLaunchKernelGGL(k_macro<float>, grid, dim3(kBlock), 0, s,
                         static_cast<const float*>(A), out, nx, pitch, plane, y0, rows);
      break;
    case LBM_FP16_OFFSET:
      hipLaunchKernelGGL(k_macro<__half>, grid, dim3(kBlock), 0, s,
                         static_cast<const __half*>(A), out, nx, pitch, plane, y0, rows);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_read(int precision, const void* A, double* out, int nx, int pitch,
                       int64_t plane, int y0, int rows, hipStream_t s) {
  const dim3 grid(unsigned((int64_t(rows) * nx + kBlock - 1) / kBlock));
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(k_read<double>, grid, dim3(kBlock), 0, s,
                         static_cast<const double*>(A), out, nx, pitch, plane, y0, rows);
      break;
    case LBM_FP32_OFFSET:
      hipLaunchKernelGGL(k_read<float>, grid, dim3(kBlock), 0, s,
                         static_cast<const float*>(A), out, nx, pitch, plane, y0, rows);
      break;
    case LBM_FP16_OFFSET:
      hipLaunchKernelGGL(k_read<__half>, grid, dim3(kBlock), 0, s,
                         static_cast<const __half*>(A), out, nx, pitch, plane, y0, rows);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_write(int precision, void* A, void* B, const double* in, int nx, int pitch,
                        int64_t plane, int y0, int rows, hipStream_t s) {
  const dim3 grid(unsigned((int64_t(rows) * nx + kBlock - 1) / kBlock));
  switch (precision) {
    case LBM_FP64:
      hipLaunchKernelGGL(k_write<double>, grid, dim3(kBlock), 0, s, static_cast<double*>(A),
                         static_cast<double*>(B), in, nx, pitch, plane, y0, rows);
      break;
    case LBM_FP32_OFFSET:
      hipLaunchKernelGGL(k_write<float>, grid, dim3(kBlock), 0, s, static_cast<float*>(A),
                         static_cast<float*>(B), in, nx, pitch, plane, y0, rows);
      break;
    case LBM_FP16_OFFSET:
      hipLaunchKernelGGL(k_write<__half>, grid, dim3(kBlock), 0, s, static_cast<__half*>(A),
                         static_cast<__half*>(B), in, nx, pitch, plane, y0, rows);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- standalone network evaluation -------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_mlp_forward(const MlpDev* w, const float* x,
                                                        float* s, int64_t n) {
  __shared__ MlpX X;
  __shared__ MlpH H;
  const int64_t r0 = int64_t(blockIdx.x) * kNnRows;
  for (int i = threadIdx.x; i < kNnRows * 32; i += kBlock) {
    const int r = i >> 5, f = i & 31;
    const int64_t row = r0 + r;
    X.x[r * kXPitch + f] = (row < n && f < 27) ? feature_bf16(w, f, x[row * 27 + f]) : 0;
  }
  __syncthreads();
  mlp_tile(w, X, H);
  for (int i = threadIdx.x; i < kNnRows * 3; i += kBlock) {
    const int r = i / 3, o = i - r * 3;
    const int64_t row = r0 + r;
    if (row < n) s[row * 3 + o] = H.o[r * 4 + o] * w->sd_out[o] + w->mu_out[o];
  }
}

hipError_t launch_mlp_forward(const MlpDev* mlp, const float* x, float* s, int64_t n,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(unsigned((n + kNnRows - 1) / kNnRows));
  hipLaunchKernelGGL(k_mlp_forward, grid, dim3(kBlock), 0, st, mlp, x, s, n);
  return hipGetLastError();
}

}  // namespace lbm
