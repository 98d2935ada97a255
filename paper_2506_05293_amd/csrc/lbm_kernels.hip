// HIP kernels of the D2Q9 time step for gfx950.
//
// One launch advances the lattice by one step (Sec. 2.1 Eq. 1 in pull form):
// every fluid node gathers the post-collision populations of its neighbours
// from buffer A (half-way bounce-back where the source is a wall or a solid,
// Eq. 12), completes the inlet / outlet column (Sec. 2.2, Sec. 3.1 Eq. 16),
// collides (Eq. 2 or MRT) and writes its post-collision populations to B.
// The same launch produces the momentum-exchange force of the step
// (Eqs. 14-15) and the mass, as per-workgroup partial sums.
//
// Grid layout (virtual block ids after the XCD remap, see xcd_remap):
//   v = 0                 reduces the partials of the previous step, in a
//                         fixed order, in FP64, into the accumulators;
//   v = 1 .. n_nn         neural outlet blocks, 64 outlet rows each;
//   v > n_nn              bulk tiles of 256 x `rows` nodes, x fastest.
//
// Memory layout: population q of node (x, y) at q*plane + y*pitch + x, with
// pitch a multiple of 64 elements; offsets f - w stored in S.
#include "d2q9_dev.hpp"
#include "lbm_internal.hpp"
#include "mlp_dev.hpp"

namespace lbm {

// Workgroups are dispatched to the eight XCDs round-robin by blockIdx; give
// each XCD a contiguous range of tiles so that the cache lines two x-adjacent
// tiles share (the pull reads one element past each tile edge) meet in the
// same L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, r = n & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Fixed-order sum of four values over the workgroup; thread 0 writes them.
template <typename T>
__device__ __forceinline__ void block_partials(T a, T b, T c, T d, T* out) {
  __shared__ T red[kBlock / 64][4];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  d = wave_sum(d);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w][0] = a;
    red[w][1] = b;
    red[w][2] = c;
    red[w][3] = d;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// Sum the per-workgroup partials of one step in FP64 and fixed order, then
// update the accumulators and the force history.
template <typename T>
__device__ void reduce_into_acc(const T* __restrict__ part, const StepLaunch& L) {
  __shared__ double red[kBlock / 64][4];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < L.nblocks; b += kBlock) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] += double(part[b * kPartials + k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = wave_sum(s[k]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) red[threadIdx.x >> 6][k] = s[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
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
}

template <typename T, int MRT>
__device__ __forceinline__ void collide(T g[9], const StepLaunch& L) {
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

// ---- bulk tile ------------------------------------------------------------------
template <typename S, int MRT>
__device__ __forceinline__ void bulk_node(const StepLaunch& L, int x, int y,
                                          typename Store<S>::T& fx, typename Store<S>::T& fy,
                                          typename Store<S>::T& dm) {
  using T = typename Store<S>::T;
  const S* __restrict__ A = static_cast<const S*>(L.A);
  S* __restrict__ B = static_cast<S*>(L.B);
  const int64_t row = int64_t(y) * L.pitch;
  uint32_t lk = 0;
  if (L.chunk[y * L.nchunk + (x >> 8)]) lk = L.links[row + x];
  if (lk & LINK_SOLID) return;
  if ((lk & LINK_OUTLET) && L.n_nn) return;   // done by the neural blocks

  int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
  if (xm < 0) xm = L.xper ? L.nx - 1 : 0;
  if (xp >= L.nx) xp = L.xper ? 0 : L.nx - 1;
  if (ym < 0) ym = L.yper ? L.ny - 1 : 0;
  if (yp >= L.ny) yp = L.yper ? 0 : L.ny - 1;
  const int64_t rm = int64_t(ym) * L.pitch, rp = int64_t(yp) * L.pitch;

  T g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int sx = cx(q) == 1 ? xm : (cx(q) == -1 ? xp : x);
    const int64_t sr = cy(q) == 1 ? rm : (cy(q) == -1 ? rp : row);
    const int64_t pull = int64_t(q) * L.plane + sr + sx;
    const int64_t back = int64_t(opp(q)) * L.plane + row + x;
    g[q] = Store<S>::ld(A + (((lk >> q) & 1u) ? back : pull));
  }
  if (lk & (LINK_INLET | LINK_OUTLET)) {
    if (lk & LINK_INLET)
      zouhe_inlet(g, L.inlet ? T(L.inlet[y]) : T(L.u_in));
    else
      zouhe_outlet(g, T(L.one_minus_rho_out));
  }
  add_force(lk, g, fx, fy);
  dm += macro(g).drho;
  collide<T, MRT>(g, L);
#pragma unroll
  for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row + x, g[q]);
}

template <typename S, int MRT>
__device__ __forceinline__ void bulk_block(const StepLaunch& L, int tile,
                                           typename Store<S>::T* part) {
  using T = typename Store<S>::T;
  const int tx = tile % L.ntx, ty = tile / L.ntx;
  const int x = tx * kChunk + threadIdx.x;
  const int yb = ty * L.rows;
  const int ye = min(yb + L.rows, L.ny);
  T fx = T(0), fy = T(0), dm = T(0);
  if (x < L.nx)
    for (int y = yb; y < ye; ++y) bulk_node<S, MRT>(L, x, y, fx, fy, dm);
  block_partials(fx, fy, dm, T(0), part);
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

template <typename S, int MRT>
__device__ void nn_block(const StepLaunch& L, int nb, typename Store<S>::T* part) {
  using T = typename Store<S>::T;
  __shared__ NnSmem<T> sm;
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
    T r[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) r[q] = g[q];
    r[3] = sm.prev[j * 4 + 0] + T(sm.u.H.o[j * 4 + 0] * w->sd_out[0] + w->mu_out[0]);
    r[6] = sm.prev[j * 4 + 1] + T(sm.u.H.o[j * 4 + 1] * w->sd_out[1] + w->mu_out[1]);
    r[7] = sm.prev[j * 4 + 2] + T(sm.u.H.o[j * 4 + 2] * w->sd_out[2] + w->mu_out[2]);
    const float drg = float(macro(r).drho);
    const bool ok = float(r[3] + wgt<T>(3)) > 0.f && float(r[6] + wgt<T>(6)) > 0.f &&
                    float(r[7] + wgt<T>(7)) > 0.f &&
                    fabsf(drg - float(sm.prev[j * 4 + 3])) < w->mass_bound;
    if (ok) {
#pragma unroll
      for (int q = 0; q < 9; ++q) g[q] = r[q];
    } else {
      zouhe_outlet(g, T(L.one_minus_rho_out));
      nfb = T(1);
    }
    dm = macro(g).drho;
    collide<T, MRT>(g, L);
    const int64_t row = int64_t(y) * L.pitch + x;
#pragma unroll
    for (int q = 0; q < 9; ++q) Store<S>::st(B + int64_t(q) * L.plane + row, g[q]);
  }
  block_partials(fx, fy, dm, nfb, part);
}

// ---- the step kernel --------------------------------------------------------------
template <typename S, int MRT>
__global__ void __launch_bounds__(kBlock) k_step(const StepLaunch L) {
  using T = typename Store<S>::T;
  const int v = xcd_remap(blockIdx.x, L.nblocks);
  T* part = static_cast<T*>(L.part_w) + kPartials * v;
  if (v == 0) {
    if (L.reduce_prev) reduce_into_acc<T>(static_cast<const T*>(L.part_r), L);
    if (threadIdx.x < kPartials) part[threadIdx.x] = T(0);
    return;
  }
  if (v <= L.n_nn) {
    nn_block<S, MRT>(L, v - 1, part);
    return;
  }
  bulk_block<S, MRT>(L, v - 1 - L.n_nn, part);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_finalize(const StepLaunch L) {
  reduce_into_acc<T>(static_cast<const T*>(L.part_r), L);
}

template <typename S, int MRT>
static hipError_t launch_step_t(const StepLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((k_step<S, MRT>), dim3(L.nblocks), dim3(kBlock), 0, s, L);
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
