// Closed-loop training of the tuning network of the characteristic outflow
// on gfx950 (C ABI of include/lbm_cbc_train.h).
//
// Sec. 4.2: segments of n_t steps start from reference states; the loss at
// step n_t is the MSE of density and velocity over the n_t columns next to
// the outlet; the network (9-20-20-2, LeakyReLU, sigmoid output maps) is
// trained on the exact gradient of that loss through the rollout.  Every
// segment runs on a strip of W = 2 n_max + 3 columns (nothing further
// upstream reaches the loss region within n_t steps), in offset form
// g = f - w, BGK collision, periodic rows, no solids.  Strips are stored
// column by column (rows fastest), so that the outlet kernels, which work
// along the rows of the last columns, read consecutive addresses.
//
// One optimiser step, every segment at once (a segment whose n_t is
// shorter than the step index sits out that step):
//   forward k = 0 .. n_max-1
//     k_fwd         outlet workgroups, one thread per outlet row: gradients
//                   of the state at the three last columns, network, LODI
//                   time derivatives (Eqs. 18-28), stored outlet state and
//                   time derivatives, and the outlet node's update (pull,
//                   outlet state by Eq. 29 and Eqs. 8-10, BGK); node
//                   workgroups, one thread per node left of the outlet
//                   column: pull streaming, BGK; the trajectory is kept;
//   k_seed          loss over Omega (its derivative with respect to the
//                   final state, the adjoint's initial value, is recomputed
//                   where the backward pass takes it);
//   backward k = n_max-1 .. 0
//     k_bwd         per node left of the last three columns: the adjoint
//                   of the post-collision state at step k+1 (the seed, or
//                   the streaming adjoint of step k+1 -- a gather:
//                   population q of node x takes the adjoint of node x + c_q),
//                   then the collision adjoint at the recomputed
//                   pre-collision state of step k+1; the two are fused
//                   because the collision adjoint at x needs only that
//                   node's adjoint (adjoints of the pulled populations
//                   alternate between two buffers);
//     k_bwd_outlet  the same node adjoints for the last three columns, plus
//                   the moment terms through which the outlet read them;
//                   then one thread per outlet row: adjoints of the outlet
//                   reconstruction, of the LODI update and of the network,
//                   the parameter gradient summed over the workgroup's 64
//                   rows from LDS (in the working precision) into a
//                   per-(segment, row block) FP64 slot;
//                   the start state's adjoint is never needed, so the
//                   streaming adjoint of step 0 is not taken;
//   k_gsum, k_lsum  first stage of the FP64 sums of the gradient and loss
//                   slots (fixed order, many workgroups);
//   k_update        second stage and Adam.
// The outlet work is latency-bound (a few rows, a long chain per row) and
// the node work bandwidth-bound, and within a step neither reads what the
// other writes.  Forward, both are workgroups of one launch (the outlet
// ones are few, hold little, and start first); backward, the outlet kernel
// holds a large LDS block through its chain and runs on a second stream
// beside the node kernel, the two joined by events after every step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "../../include/lbm_cbc_train.h"
#include "d2q9_dev.hpp"
#include "lbm_internal.hpp"

namespace lbm {
namespace {

constexpr int kNP = LBM_CBC_NPARAMS;        // the tuning network (2 outputs)
constexpr int kNPNn = LBM_NN9_NPARAMS;      // the Eq. 16 network (3 outputs)
constexpr int kNPMax = kNPNn;               // stride of the gradient slots
constexpr int kIn = 9, kH = 20;
constexpr int kOW1 = 0, kOB1 = kH * kIn, kOW2 = kOB1 + kH, kOB2 = kOW2 + kH * kH,
              kOW3 = kOB2 + kH, kOB3 = kOW3 + 2 * kH, kOB3n = kOW3 + 3 * kH;
static_assert(kOB3 + 2 == kNP, "parameter count");
static_assert(kOB3n + 3 == kNPNn, "parameter count");
constexpr int kRows = 64;            // outlet rows per workgroup (one wave)
constexpr int kNodes = 256;          // nodes per workgroup
// The backward outlet workgroup is one wave: it takes the node adjoints of
// the last three columns of its 64 rows, then the rows, then the
// parameter-gradient sums.  It runs beside the bulk kernel, so the fewer CU
// slots it holds through its long row chain the better (four waves, one per
// column and all sharing the sums, measured 1 % slower per optimiser step).
constexpr int kBwdThreads = kRows;
// The step-to-step events only order the two streams of one device: no
// system-scope fence (measured 3 % faster per optimiser step).
constexpr unsigned kEventFlags = hipEventDisableTiming | hipEventDisableSystemFence;
constexpr int kMaxSteps = 64;
constexpr int kMadj = 12;            // per outlet row: 3 columns x (drho, u, v) + y-part
                                     // (Eq. 16 outlet: the 9 population adjoints it left)
// The outlet of a segment: the characteristic outflow with its tuning
// network, or the reconstruction of Eq. 16 with its network.
constexpr int kOutCbc = 0, kOutNn = 1;

struct CtState {
  float w[kNPMax];                   // FP32 masters
  double m[kNPMax], v[kNPMax];       // Adam moments
  double mu[kIn], sd[kIn];           // input standardisation
  double leaky, sig_scale, sig_shift, kap_scale, kap_shift;
  double mu_out[3], sd_out[3];       // Eq. 16: s = o sd_out + mu_out
  double rho_inf_m1;                 // rho_inf - 1
  double loss;
  double grad[kNPMax];
};

template <typename T>
struct CtArgs {
  T* traj;              // [seg][n_max+1][9][W][ny] (rows fastest)
  T* outs;              // [seg][n_max][ny][3]    outlet state drho', u', v'
                        //                        (Eq. 16: the reconstructed g3, g6, g7)
  T* dts;               // [seg][n_max+1][ny][3]  c_s^2 rho_t, u_t, v_t
  T* lamF[2];           // [seg][9][W][ny] each   adjoint of the pulled populations,
                        //                        step k in buffer k & 1
  T* lamP;              // [seg][ny][3]           adjoint of the time derivatives
  T* madj[2];           // [seg][ny][12] each     moment adjoints from the outlet,
                        //                        step k in buffer k & 1
  const T* ref;         // [seg][3][ny][n_max]    rho - 1, u, v
  const int* nts;       // [seg]
  double* gslot;        // [seg][nrb][kNPMax]
  double* lslot;        // [seg][nlb]
  CtState* st;
  int ny, W, n_max, nrb, nlb;
  int nlb_fwd, nlb_bwd;  // node blocks of the bulk kernels (columns 0..W-2, 0..W-4)
  int nrb_fwd, n_seg;    // outlet blocks of the forward kernel (256 rows each), segments
  int64_t plane;        // ny * W; node (x, y) of a plane at x * ny + y
  const double* seg_omega;   // [seg] 1 / tau
  const double* seg_k1c;     // [seg] (1 - M^2) c_s / L  (kappa_1 = sigma k1c)
  double seg_scale;     // 1 / n_seg
};

template <typename T>
__device__ __forceinline__ T* state_at(const CtArgs<T>& a, int s, int k) {
  return a.traj + (int64_t(s) * (a.n_max + 1) + k) * 9 * a.plane;
}

__device__ __forceinline__ int wrap(int y, int ny) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); }

template <typename T>
__device__ __forceinline__ T leaky(T x, T a) {
  return x > T(0) ? x : a * x;
}

template <typename T>
__device__ __forceinline__ T tanh_t(T x) {
  if constexpr (sizeof(T) == 8)
    return tanh(x);
  else
    return tanhf(x);
}

template <typename T>
__device__ __forceinline__ T sigmoid(T s) {
  if constexpr (sizeof(T) == 8)
    return T(1) / (T(1) + exp(-s));
  else
    return T(1) / (T(1) + expf(-s));
}

template <typename T>
__device__ __forceinline__ void load_node(const T* A, int64_t plane, int64_t idx, T g[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) g[q] = A[q * plane + idx];
}

template <typename T>
__device__ __forceinline__ void node_state(const T* A, int64_t plane, int64_t idx, T& drho, T& u,
                                           T& v) {
  T g[9];
  load_node(A, plane, idx, g);
  const Macro<T> m = macro(g);
  drho = m.drho;
  u = m.jx / m.rho;
  v = m.jy / m.rho;
}

// Pull streaming into node (x, y) of the strip: sources left of the strip
// are replaced by the edge column itself, the outlet's unknowns are left 0.
template <typename T>
__device__ __forceinline__ void pull(const T* A, int64_t plane, int W, int ny, int x, int y,
                                     T g[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int sx = x - cx(q);
    const int sy = wrap(y - cy(q), ny);
    if (sx < 0) sx = x;
    g[q] = sx <= W - 1 ? A[q * plane + int64_t(sx) * ny + sy] : T(0);
  }
}

// State and gradients at the outlet node of row r (columns W-3 .. W-1):
// second-order one-sided in x, central in y (periodic rows).
template <typename T>
struct OutIn {
  T drho, u, v;
  T g[6];      // p_x, u_x, v_x, p_y, u_y, v_y
};

template <typename T>
__device__ OutIn<T> outlet_inputs(const T* A, int64_t plane, int W, int ny, int r) {
  const T cs2 = T(1.0 / 3.0);
  T d[3], uu[3], vv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) node_state(A, plane, int64_t(W - 3 + c) * ny + r, d[c], uu[c], vv[c]);
  T dn, un, vn, ds, us, vs;
  node_state(A, plane, int64_t(W - 1) * ny + wrap(r + 1, ny), dn, un, vn);
  node_state(A, plane, int64_t(W - 1) * ny + wrap(r - 1, ny), ds, us, vs);
  OutIn<T> o;
  o.drho = d[2];
  o.u = uu[2];
  o.v = vv[2];
  o.g[0] = cs2 * (T(0.5) * (T(3) * d[2] - T(4) * d[1] + d[0]));
  o.g[1] = T(0.5) * (T(3) * uu[2] - T(4) * uu[1] + uu[0]);
  o.g[2] = T(0.5) * (T(3) * vv[2] - T(4) * vv[1] + vv[0]);
  o.g[3] = cs2 * (T(0.5) * (dn - ds));
  o.g[4] = T(0.5) * (un - us);
  o.g[5] = T(0.5) * (vn - vs);
  return o;
}

// The isothermal LODI update (Eqs. 18-26, L_1 of Eqs. 27-28, T_1,exact = 0).
template <typename T>
struct Lodi {
  T rho, p, L1, L3, L5, T1, T3, T5, rho_t, u_t, v_t;
};

template <typename T>
__device__ Lodi<T> lodi(const OutIn<T>& in, T sigma, T kappa2, T k1c, const CtState* st) {
  const T cs2 = T(1.0 / 3.0), cs = T(0.57735026918962576451);
  const T px = in.g[0], ux = in.g[1], vx = in.g[2], py = in.g[3], uy = in.g[4], vy = in.g[5];
  const T u = in.u, v = in.v;
  Lodi<T> l;
  l.rho = T(1) + in.drho;
  l.p = cs2 * l.rho;
  l.L3 = u * vx;
  l.L5 = (u + cs) * (px + l.rho * cs * ux);
  l.T1 = -(v * py + l.p * vy - l.rho * cs * v * uy);
  l.T3 = -(v * vy + py / l.rho);
  l.T5 = -(v * py + l.p * vy + l.rho * cs * v * uy);
  l.L1 = sigma * k1c * cs2 * (in.drho - T(st->rho_inf_m1)) - kappa2 * l.T1 + l.T1;
  l.rho_t = (-(l.L5 + l.L1) + (l.T5 + l.T1)) / (T(2) * cs2);
  l.u_t = (-(l.L5 - l.L1) + (l.T5 - l.T1)) / (T(2) * l.rho * cs);
  l.v_t = -l.L3 + l.T3;
  return l;
}

// ---- forward -------------------------------------------------------------------------
// The weights (662 or 683) are read by every row: staged once per
// workgroup in LDS (uniform reads, no scalar-load latency inside the layers).
__device__ __forceinline__ void stage_weights(const CtState* st, float* sw, int nthreads,
                                              int np = kNP) {
  for (int i = threadIdx.x; i < np; i += nthreads) sw[i] = st->w[i];
  __syncthreads();
}

// The outlet row r of segment s at step k: every global load of the row is
// issued before the weights are staged, so the two overlap (rows past the
// end read the last row and store nothing).  Called by every thread of the
// workgroup (the staging synchronises it).
template <typename T>
__device__ __forceinline__ void fwd_outlet_row(const CtArgs<T>& a, float* sw, int s, int k, int r) {
  const CtState* st = a.st;
  const bool valid = r < a.ny;
  const int rl = valid ? r : a.ny - 1;
  const OutIn<T> in = outlet_inputs(state_at(a, s, k), a.plane, a.W, a.ny, rl);
  const T* P = a.dts + ((int64_t(s) * (a.n_max + 1) + k) * a.ny + rl) * 3;
  const T prev[3] = {P[0], P[1], P[2]};
  stage_weights(st, sw, kNodes);
  if (!valid) return;
  T z[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) {
    const T f = i < 6 ? in.g[i] : prev[i - 6];
    z[i] = (f - T(st->mu[i])) / T(st->sd[i]);
  }
  const T sl = T(st->leaky);
  T h1[kH];
#pragma unroll
  for (int o = 0; o < kH; ++o) {
    T acc = T(sw[kOB1 + o]);
#pragma unroll
    for (int i = 0; i < kIn; ++i) acc += T(sw[kOW1 + o * kIn + i]) * z[i];
    h1[o] = leaky(acc, sl);
  }
  T s0 = T(sw[kOB3]), s1 = T(sw[kOB3 + 1]);
#pragma unroll 1
  for (int o = 0; o < kH; ++o) {
    T acc = T(sw[kOB2 + o]);
#pragma unroll
    for (int m = 0; m < kH; ++m) acc += T(sw[kOW2 + o * kH + m]) * h1[m];
    const T h = leaky(acc, sl);
    s0 += T(sw[kOW3 + o]) * h;
    s1 += T(sw[kOW3 + kH + o]) * h;
  }
  const T sigma = T(st->sig_scale) * sigmoid(s0) + T(st->sig_shift);
  const T kappa2 = T(st->kap_scale) * sigmoid(s1) + T(st->kap_shift);
  const Lodi<T> l = lodi(in, sigma, kappa2, T(a.seg_k1c[s]), st);
  T* o = a.outs + ((int64_t(s) * a.n_max + k) * a.ny + r) * 3;
  o[0] = in.drho + l.rho_t;                 // forward Euler
  o[1] = in.u + l.u_t;
  o[2] = in.v + l.v_t;
  T* Pn = a.dts + ((int64_t(s) * (a.n_max + 1) + k + 1) * a.ny + r) * 3;
  Pn[0] = T(1.0 / 3.0) * l.rho_t;
  Pn[1] = l.u_t;
  Pn[2] = l.v_t;
  // the outlet node itself: pull, completed by the new outlet state
  // (Eq. 29, Eqs. 8-10), BGK
  T g[9];
  const int64_t n = int64_t(a.W - 1) * a.ny + r;
  pull(state_at(a, s, k), a.plane, a.W, a.ny, a.W - 1, r, g);
  outlet_state(g, in.drho + l.rho_t, in.u + l.u_t, in.v + l.v_t);
  collide_bgk(g, T(a.seg_omega[s]));
  T* B = state_at(a, s, k + 1);
#pragma unroll
  for (int q = 0; q < 9; ++q) B[q * a.plane + n] = g[q];
}

// The outlet row r with the reconstruction of Eq. 16: the pulled offsets
// of column L-1 = W-2 are the network's features (standardised), the
// unknowns are g_i = f_i(L-1) + s_i for i = 3, 6, 7 with s = o sd_out +
// mu_out, o the 9-20-20-3 network (tanh hidden layers, linear output).
template <typename T>
__device__ __forceinline__ void fwd_outlet_row_nn(const CtArgs<T>& a, float* sw, int s, int k,
                                                  int r) {
  const CtState* st = a.st;
  const bool valid = r < a.ny;
  const int rl = valid ? r : a.ny - 1;
  const T* A = state_at(a, s, k);
  T fe[9], g[9];
  pull(A, a.plane, a.W, a.ny, a.W - 2, rl, fe);
  pull(A, a.plane, a.W, a.ny, a.W - 1, rl, g);
  stage_weights(st, sw, kNodes, kNPNn);
  if (!valid) return;
  T z[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) z[i] = (fe[i] - T(st->mu[i])) / T(st->sd[i]);
  T h1[kH];
#pragma unroll
  for (int o = 0; o < kH; ++o) {
    T acc = T(sw[kOB1 + o]);
#pragma unroll
    for (int i = 0; i < kIn; ++i) acc += T(sw[kOW1 + o * kIn + i]) * z[i];
    h1[o] = tanh_t(acc);
  }
  T o0 = T(sw[kOB3n]), o1 = T(sw[kOB3n + 1]), o2 = T(sw[kOB3n + 2]);
#pragma unroll 1
  for (int o = 0; o < kH; ++o) {
    T acc = T(sw[kOB2 + o]);
#pragma unroll
    for (int m = 0; m < kH; ++m) acc += T(sw[kOW2 + o * kH + m]) * h1[m];
    const T h = tanh_t(acc);
    o0 += T(sw[kOW3 + o]) * h;
    o1 += T(sw[kOW3 + kH + o]) * h;
    o2 += T(sw[kOW3 + 2 * kH + o]) * h;
  }
  g[3] = fe[3] + (o0 * T(st->sd_out[0]) + T(st->mu_out[0]));
  g[6] = fe[6] + (o1 * T(st->sd_out[1]) + T(st->mu_out[1]));
  g[7] = fe[7] + (o2 * T(st->sd_out[2]) + T(st->mu_out[2]));
  T* O = a.outs + ((int64_t(s) * a.n_max + k) * a.ny + r) * 3;
  O[0] = g[3];
  O[1] = g[6];
  O[2] = g[7];
  collide_bgk(g, T(a.seg_omega[s]));
  T* B = state_at(a, s, k + 1);
  const int64_t n = int64_t(a.W - 1) * a.ny + r;
#pragma unroll
  for (int q = 0; q < 9; ++q) B[q * a.plane + n] = g[q];
}

template <typename T, int OK>
__device__ __forceinline__ void pre_collision(const CtArgs<T>& a, int s, int k, int x, int y,
                                              T g[9]) {
  pull(state_at(a, s, k), a.plane, a.W, a.ny, x, y, g);
  if (x == a.W - 1) {
    const T* o = a.outs + ((int64_t(s) * a.n_max + k) * a.ny + y) * 3;
    if constexpr (OK == kOutNn) {
      g[3] = o[0];                          // Eq. 16
      g[6] = o[1];
      g[7] = o[2];
    } else {
      outlet_state(g, o[0], o[1], o[2]);    // Eq. 29, Eqs. 8-10
    }
  }
}

// One forward step: the first n_seg * nrb_fwd workgroups take the outlet
// rows (256 per workgroup; their network chain is long but they are few and
// start first), the rest every node left of the outlet column.
template <typename T, int OK>
__global__ void __launch_bounds__(kNodes) k_fwd(const CtArgs<T> a, int k) {
  __shared__ float sw[kNPMax];
  int b = int(blockIdx.x);
  const int nout = a.n_seg * a.nrb_fwd;
  if (b < nout) {
    const int s = b / a.nrb_fwd;
    if (k >= a.nts[s]) return;                   // uniform over the workgroup
    const int r = (b - s * a.nrb_fwd) * kNodes + int(threadIdx.x);
    if constexpr (OK == kOutNn)
      fwd_outlet_row_nn(a, sw, s, k, r);
    else
      fwd_outlet_row(a, sw, s, k, r);
    return;
  }
  b -= nout;
  const int s = b / a.nlb_fwd;
  if (k >= a.nts[s]) return;
  const int64_t n = int64_t(b - s * a.nlb_fwd) * kNodes + threadIdx.x;
  if (n >= a.plane - a.ny) return;
  const int x = int(n / a.ny), y = int(n - int64_t(x) * a.ny);
  T g[9];
  pre_collision<T, OK>(a, s, k, x, y, g);
  collide_bgk(g, T(a.seg_omega[s]));
  T* B = state_at(a, s, k + 1);
#pragma unroll
  for (int q = 0; q < 9; ++q) B[q * a.plane + n] = g[q];
}

// ---- loss and the adjoint's initial value ------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// The loss term of node (x, y) of segment s (0 outside Omega, the last n_t
// columns) and its derivative with respect to the node's final state, the
// adjoint's initial value: with e = rho - rho_ref, u - u_ref, v - v_ref and
// c = 1 / (n_seg n_t ny), loss = c (e_rho^2 + |e_u|^2) and
// lam_q = 2 c (e_rho + (e_u . (c_q - u)) / rho).
template <typename T>
__device__ __forceinline__ double seed_adjoint(const CtArgs<T>& a, int s, int nt, int x, int y,
                                               int64_t n, T lam[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) lam[q] = T(0);
  if (x < a.W - nt) return 0.0;
  T drho, u, v;
  node_state(state_at(a, s, nt), a.plane, n, drho, u, v);
  const int e = x - (a.W - a.n_max);                      // reference entry of column x
  const T* R = a.ref + (int64_t(s) * 3 * a.ny + y) * a.n_max + e;
  const int64_t cstride = int64_t(a.ny) * a.n_max;
  const T er = drho - R[0], eu = u - R[cstride], ev = v - R[2 * cstride];
  const double c = a.seg_scale / (double(nt) * double(a.ny));
  const T c2 = T(2.0 * c), inv = T(1) / (T(1) + drho);
#pragma unroll
  for (int q = 0; q < 9; ++q) lam[q] = c2 * (er + (eu * (T(cx(q)) - u) + ev * (T(cy(q)) - v)) * inv);
  return c * (double(er) * double(er) + double(eu) * double(eu) + double(ev) * double(ev));
}

// The loss over Omega of every segment (per-workgroup FP64 slots) and the
// zero adjoint of the time derivatives; the adjoint's initial value is
// recomputed where the backward pass starts.
template <typename T>
__global__ void __launch_bounds__(kNodes) k_seed(const CtArgs<T> a) {
  __shared__ double sh[kNodes / 64];
  const int s = blockIdx.y;
  const int nt = a.nts[s];
  const int64_t n = int64_t(blockIdx.x) * kNodes + threadIdx.x;
  double contrib = 0.0;
  if (n < a.plane) {
    const int x = int(n / a.ny), y = int(n - int64_t(x) * a.ny);
    T lam[9];
    contrib = seed_adjoint(a, s, nt, x, y, n, lam);
    if (n < int64_t(a.ny) * 3) a.lamP[int64_t(s) * a.ny * 3 + n] = T(0);
  }
  const double t = block_sum(contrib, sh);
  if (threadIdx.x == 0) a.lslot[int64_t(s) * a.nlb + blockIdx.x] = t;
}

// ---- backward --------------------------------------------------------------------------
// BGK: A = f - omega (f - f^eq(rho, j)), so with
//   d f_i^eq / d rho = w_i (1 - 9/2 (c_i.u)^2 + 3/2 u.u),
//   d f_i^eq / d j   = w_i (3 c_i + 9 (c_i.u) c_i - 3 u),
// lam_f_j = (1 - omega) lam_j + omega (Lambda_rho + c_j . Lambda_j), Lambda the
// lam-weighted sums of those derivatives.
// Adjoint of the post-collision state A_kk at node (x, y) from the adjoints
// LF of the populations pulled at step kk (streaming adjoint) and the moment
// adjoints the outlet left for the last three columns.
template <typename T, int OK>
__device__ __forceinline__ void state_adjoint(const CtArgs<T>& a, int s, int kk, int x, int y,
                                              int64_t n, const T* LF, T lam[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int dx = x + cx(q);
    const int dy = wrap(y + cy(q), a.ny);
    T l = T(0);
    if (dx >= 0 && dx <= a.W - 1) l = LF[q * a.plane + int64_t(dx) * a.ny + dy];
    if (x == 0 && cx(q) == 1) l += LF[q * a.plane + dy];                  // edge copies
    lam[q] = l;
  }
  if (OK == kOutNn && x >= a.W - 3) {
    // Eq. 16 read population q of this node as feature q of the outlet row
    // r = y + c_y(q) (a pull into column W-2) -- and, for q = 3, 6, 7, as
    // f_q(L-1) of that row's reconstruction: the row left both adjoints in
    // its slot q
    const T* MA = a.madj[kk & 1] + int64_t(s) * a.ny * kMadj;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      if (x == a.W - 2 - cx(q)) lam[q] += MA[int64_t(wrap(y + cy(q), a.ny)) * kMadj + q];
  } else if (x >= a.W - 3) {
    const int c = x - (a.W - 3);
    const T* MA = a.madj[kk & 1] + int64_t(s) * a.ny * kMadj;
    const T* M = MA + int64_t(y) * kMadj;
    T ld = M[3 * c], lu = M[3 * c + 1], lv = M[3 * c + 2];
    if (c == 2) {
      const T* Ms = MA + int64_t(wrap(y - 1, a.ny)) * kMadj;   // row y = r + 1
      const T* Mn = MA + int64_t(wrap(y + 1, a.ny)) * kMadj;   // row y = r - 1
      ld += Ms[9] - Mn[9];
      lu += Ms[10] - Mn[10];
      lv += Ms[11] - Mn[11];
    }
    T drho, u, v;
    node_state(state_at(a, s, kk), a.plane, n, drho, u, v);
    const T inv = T(1) / (T(1) + drho);
#pragma unroll
    for (int q = 0; q < 9; ++q) lam[q] += ld + (lu * (T(cx(q)) - u) + lv * (T(cy(q)) - v)) * inv;
  }
}

// Adjoint of the pulled populations of node (x, y) at step k (lf): the
// adjoint of the post-collision state at step k+1 (the seed at the last
// step), then the collision adjoint at the recomputed pre-collision state.
template <typename T, int OK>
__device__ __forceinline__ void node_adjoint(const CtArgs<T>& a, int s, int nt, int k, int x, int y,
                                             int64_t n, T lf[9]) {
  const int64_t so = int64_t(s) * 9 * a.plane;
  T lam[9];
  if (k + 1 == nt) {
    (void)seed_adjoint(a, s, nt, x, y, n, lam);
  } else {
    state_adjoint<T, OK>(a, s, k + 1, x, y, n, a.lamF[(k + 1) & 1] + so, lam);
  }
  T g[9];
  pre_collision<T, OK>(a, s, k, x, y, g);
  const Macro<T> m = macro(g);
  const T u = m.jx / m.rho, v = m.jy / m.rho;
  const T usq = T(1.5) * (u * u + v * v);
  T Lr = T(0), Ljx = T(0), Ljy = T(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const T cu = T(cx(q)) * u + T(cy(q)) * v;
    const T wl = wgt<T>(q) * lam[q];
    Lr += wl * (T(1) - T(4.5) * cu * cu + usq);
    Ljx += wl * (T(3 * cx(q)) + T(9) * cu * T(cx(q)) - T(3) * u);
    Ljy += wl * (T(3 * cy(q)) + T(9) * cu * T(cy(q)) - T(3) * v);
  }
  const T om = T(a.seg_omega[s]);
#pragma unroll
  for (int q = 0; q < 9; ++q)
    lf[q] = (T(1) - om) * lam[q] + om * (Lr + T(cx(q)) * Ljx + T(cy(q)) * Ljy);
}

// Every node left of the last three columns (whose adjoints need the
// outlet's moment adjoints: the outlet kernel takes those).
template <typename T, int OK>
__global__ void __launch_bounds__(kNodes) k_bwd(const CtArgs<T> a, int k) {
  const int s = blockIdx.y;
  const int nt = a.nts[s];
  if (k >= nt) return;
  const int64_t n = int64_t(blockIdx.x) * kNodes + threadIdx.x;
  if (n >= a.plane - 3 * int64_t(a.ny)) return;
  const int x = int(n / a.ny), y = int(n - int64_t(x) * a.ny);
  T lf[9];
  node_adjoint<T, OK>(a, s, nt, k, x, y, n, lf);
  T* LF = a.lamF[k & 1] + int64_t(s) * 9 * a.plane;
#pragma unroll
  for (int q = 0; q < 9; ++q) LF[q * a.plane + n] = lf[q];
}

// Per-row arrays, read row by row in the gradient sums and one row per lane
// in the row work: rows of an odd number of words keep the lanes of the
// latter on distinct banks.
constexpr int kHp = kH + 1;
template <typename T>
struct alignas(16) BwdSmem {
  T z[kRows][kIn];
  T h1[kRows][kHp];
  T h2[kRows][kHp];
  T d1[kRows][kHp];   // adjoint of the first pre-activation
  T d2[kRows][kHp];   // adjoint of the second pre-activation
  T ds[kRows][3];     // adjoint of s_0, s_1
};

// Sum over the workgroup's rows with four independent accumulators (a fixed
// order: rows r, r + 4, ... in each, then the four in pairs).
template <typename F>
__device__ __forceinline__ auto sum_rows(F f) {
  decltype(f(0)) a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 4
  for (int rr = 0; rr < kRows; rr += 4) {
    a0 += f(rr);
    a1 += f(rr + 1);
    a2 += f(rr + 2);
    a3 += f(rr + 3);
  }
  return (a0 + a1) + (a2 + a3);
}

template <typename T>
// The node adjoints of the outlet column and of the two columns before it
// for the workgroup's 64 rows (with several waves, one column each), then
// the outlet rows on the first wave; every thread stages the weights and
// shares the parameter-gradient sums.
__global__ void __launch_bounds__(kBwdThreads) k_bwd_outlet(const CtArgs<T> a, int k) {
  __shared__ BwdSmem<T> sm;
  __shared__ float sw[kNP];
  const int s = blockIdx.y;
  const int nt = a.nts[s];
  if (k >= nt) return;                           // uniform over the workgroup
  const int j = threadIdx.x;
  const int wv = j / kRows;
  const bool rowt = wv == 0;
  const int r = blockIdx.x * kRows + (j & (kRows - 1));
  const CtState* st = a.st;
  const T cs2 = T(1.0 / 3.0), cs = T(0.57735026918962576451);
  // every global load of the row is issued before the weights are staged
  // (rows past the end read the last row and contribute nothing)
  const bool valid = rowt && r < a.ny;
  const int rl = r < a.ny ? r : a.ny - 1;
  T* LF = a.lamF[k & 1] + int64_t(s) * 9 * a.plane;
  T* LP = a.lamP + (int64_t(s) * a.ny + rl) * 3;
  const int64_t on = int64_t(a.W - 1) * a.ny + rl;
  OutIn<T> in{};
  T prev[3] = {T(0), T(0), T(0)}, lp[3] = {T(0), T(0), T(0)}, lf[9];
  T d1 = T(0), u1 = T(0), v1 = T(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) lf[q] = T(0);
  // the outlet column's adjoint stays in wave 0's registers for the outlet
#pragma unroll
  for (int c = wv; c < 3; c += kBwdThreads / kRows) {
    if (r < a.ny) {
      const int x = a.W - 1 - c;
      const int64_t n = int64_t(x) * a.ny + r;
      T l9[9];
      node_adjoint<T, kOutCbc>(a, s, nt, k, x, r, n, l9);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        if (c == 0) lf[q] = l9[q];
        else LF[q * a.plane + n] = l9[q];
      }
    }
  }
  if (rowt) {
    in = outlet_inputs(state_at(a, s, k), a.plane, a.W, a.ny, rl);
    const T* P = a.dts + ((int64_t(s) * (a.n_max + 1) + k) * a.ny + rl) * 3;
    const T* o3 = a.outs + ((int64_t(s) * a.n_max + k) * a.ny + rl) * 3;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      prev[i] = P[i];
      lp[i] = LP[i];
    }
    d1 = o3[0];
    u1 = o3[1];
    v1 = o3[2];
  }
  stage_weights(st, sw, kBwdThreads);
  if (valid) {
    // recompute the forward of this row
    T z[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) {
      const T f = i < 6 ? in.g[i] : prev[i - 6];
      z[i] = (f - T(st->mu[i])) / T(st->sd[i]);
      sm.z[j][i] = z[i];
    }
    const T sl = T(st->leaky);
    // activations and LeakyReLU slopes live in LDS (the slopes are scaled
    // into adjoints below), which keeps the FP64 variant within registers
#pragma unroll 1
    for (int o = 0; o < kH; ++o) {
      T acc = T(sw[kOB1 + o]);
#pragma unroll
      for (int i = 0; i < kIn; ++i) acc += T(sw[kOW1 + o * kIn + i]) * z[i];
      sm.h1[j][o] = leaky(acc, sl);
      sm.d1[j][o] = acc > T(0) ? T(1) : sl;
    }
    T s0 = T(sw[kOB3]), s1 = T(sw[kOB3 + 1]);
#pragma unroll 1
    for (int o = 0; o < kH; ++o) {
      T acc = T(sw[kOB2 + o]);
#pragma unroll 4
      for (int m = 0; m < kH; ++m) acc += T(sw[kOW2 + o * kH + m]) * sm.h1[j][m];
      const T h = leaky(acc, sl);
      sm.h2[j][o] = h;
      sm.d2[j][o] = acc > T(0) ? T(1) : sl;     // slope, scaled below
      s0 += T(sw[kOW3 + o]) * h;
      s1 += T(sw[kOW3 + kH + o]) * h;
    }
    const T sg0 = sigmoid(s0), sg1 = sigmoid(s1);
    const T sigma = T(st->sig_scale) * sg0 + T(st->sig_shift);
    const T kappa2 = T(st->kap_scale) * sg1 + T(st->kap_shift);
    const Lodi<T> l = lodi(in, sigma, kappa2, T(a.seg_k1c[s]), st);
    const T rho1 = T(1) + d1;

    // outlet reconstruction (offset form: g0 = drho' (1 + u') + u' - (g2 + g4)
    // - 2 (g1 + g5 + g8), g3 = g1 - 2/3 rho' u', g6 = g8 + (g4 - g2)/2 - rho' u'/6
    // + rho' v'/2, g7 = g5 - (g4 - g2)/2 - rho' u'/6 - rho' v'/2)
    const T ld1 = lf[0] * (T(1) + u1) - lf[3] * T(2.0 / 3.0) * u1 +
                  lf[6] * (-u1 / T(6) + T(0.5) * v1) + lf[7] * (-u1 / T(6) - T(0.5) * v1);
    const T lu1 = rho1 * (lf[0] - T(2.0 / 3.0) * lf[3] - lf[6] / T(6) - lf[7] / T(6));
    const T lv1 = rho1 * T(0.5) * (lf[6] - lf[7]);
    LF[0 * a.plane + on] = T(0);
    LF[1 * a.plane + on] = lf[1] - T(2) * lf[0] + lf[3];
    LF[2 * a.plane + on] = lf[2] - lf[0] - T(0.5) * lf[6] + T(0.5) * lf[7];
    LF[3 * a.plane + on] = T(0);
    LF[4 * a.plane + on] = lf[4] - lf[0] + T(0.5) * lf[6] - T(0.5) * lf[7];
    LF[5 * a.plane + on] = lf[5] - T(2) * lf[0] + lf[7];
    LF[6 * a.plane + on] = T(0);
    LF[7 * a.plane + on] = T(0);
    LF[8 * a.plane + on] = lf[8] - T(2) * lf[0] + lf[6];

    // forward Euler and the stored time derivatives
    const T lrt = ld1 + cs2 * lp[0], lut = lu1 + lp[1], lvt = lv1 + lp[2];
    T ldr = ld1, lu = lu1, lv = lv1;             // centre state
    T lg[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};

    // LODI (Eqs. 18-28)
    const T rho = l.rho, u = in.u, v = in.v;
    const T px = in.g[0], ux = in.g[1], vx = in.g[2], py = in.g[3], uy = in.g[4], vy = in.g[5];
    const T ia = T(1) / (T(2) * cs2), ib = T(1) / (T(2) * rho * cs);
    const T lL5 = -ia * lrt - ib * lut;
    const T lL1 = -ia * lrt + ib * lut;
    const T lT5 = ia * lrt + ib * lut;
    T lT1 = ia * lrt - ib * lut;
    ldr += -(l.u_t / rho) * lut;
    const T lL3 = -lvt, lT3 = lvt;
    const T k1c = T(a.seg_k1c[s]);
    const T lsig = lL1 * k1c * cs2 * (in.drho - T(st->rho_inf_m1));
    ldr += lL1 * sigma * k1c * cs2;
    const T lkap = -lL1 * l.T1;
    lT1 += (T(1) - kappa2) * lL1;
    // L_3 = u v_x
    lu += lL3 * vx;
    lg[2] += lL3 * u;
    // L_5 = (u + c_s)(p_x + rho c_s u_x)
    lu += lL5 * (px + rho * cs * ux);
    lg[0] += lL5 * (u + cs);
    ldr += lL5 * (u + cs) * cs * ux;
    lg[1] += lL5 * (u + cs) * rho * cs;
    // T_1 = -(v p_y + p v_y - rho c_s v u_y)
    lv += lT1 * (-py + rho * cs * uy);
    lg[3] += -lT1 * v;
    ldr += lT1 * (-cs2 * vy + cs * v * uy);
    lg[5] += -lT1 * l.p;
    lg[4] += lT1 * rho * cs * v;
    // T_5 = -(v p_y + p v_y + rho c_s v u_y)
    lv += lT5 * (-py - rho * cs * uy);
    lg[3] += -lT5 * v;
    ldr += lT5 * (-cs2 * vy - cs * v * uy);
    lg[5] += -lT5 * l.p;
    lg[4] += -lT5 * rho * cs * v;
    // T_3 = -(v v_y + p_y / rho)
    lv += -lT3 * vy;
    lg[5] += -lT3 * v;
    lg[3] += -lT3 / rho;
    ldr += lT3 * py / (rho * rho);

    // network: output maps, then the two hidden layers
    const T ds0 = lsig * T(st->sig_scale) * sg0 * (T(1) - sg0);
    const T ds1 = lkap * T(st->kap_scale) * sg1 * (T(1) - sg1);
    sm.ds[j][0] = ds0;
    sm.ds[j][1] = ds1;
#pragma unroll
    for (int o = 0; o < kH; ++o)
      sm.d2[j][o] *= T(sw[kOW3 + o]) * ds0 + T(sw[kOW3 + kH + o]) * ds1;
    T lz[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) lz[i] = T(0);
#pragma unroll 1
    for (int m = 0; m < kH; ++m) {
      T acc = T(0);
#pragma unroll
      for (int o = 0; o < kH; ++o) acc += T(sw[kOW2 + o * kH + m]) * sm.d2[j][o];
      const T d = acc * sm.d1[j][m];
      sm.d1[j][m] = d;
#pragma unroll
      for (int i = 0; i < kIn; ++i) lz[i] += T(sw[kOW1 + m * kIn + i]) * d;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) lg[i] += lz[i] / T(st->sd[i]);
#pragma unroll
    for (int i = 0; i < 3; ++i) LP[i] = lz[6 + i] / T(st->sd[6 + i]);

    // gradients -> moments of the three columns
    T* M = a.madj[k & 1] + (int64_t(s) * a.ny + r) * kMadj;
    M[0] = T(0.5) * cs2 * lg[0];
    M[1] = T(0.5) * lg[1];
    M[2] = T(0.5) * lg[2];
    M[3] = T(-2) * cs2 * lg[0];
    M[4] = T(-2) * lg[1];
    M[5] = T(-2) * lg[2];
    M[6] = ldr + T(1.5) * cs2 * lg[0];
    M[7] = lu + T(1.5) * lg[1];
    M[8] = lv + T(1.5) * lg[2];
    M[9] = T(0.5) * cs2 * lg[3];
    M[10] = T(0.5) * lg[4];
    M[11] = T(0.5) * lg[5];
  } else if (rowt) {
#pragma unroll
    for (int i = 0; i < kIn; ++i) sm.z[j][i] = T(0);
#pragma unroll
    for (int o = 0; o < kH; ++o) sm.h1[j][o] = sm.h2[j][o] = sm.d1[j][o] = sm.d2[j][o] = T(0);
    sm.ds[j][0] = sm.ds[j][1] = T(0);
  }
  __syncthreads();
  // parameter gradient of the workgroup's rows, summed in the working
  // precision (FP64 in the FP64 variant: 0.1 ms per optimiser step less in
  // FP32) and added to its FP64 slot (the slot values are all requested
  // before the sums, so their latency overlaps)
  double* G = a.gslot + (int64_t(s) * a.nrb + blockIdx.x) * kNPMax;
  constexpr int kPer = (kNP + kBwdThreads - 1) / kBwdThreads;
  double old[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int p = j + u * kBwdThreads;
    old[u] = p < kNP ? G[p] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int p = j + u * kBwdThreads;
    if (p >= kNP) break;
    T acc;
    if (p < kOB1) {
      const int m = p / kIn, i = p - m * kIn;
      acc = sum_rows([&](int rr) { return sm.d1[rr][m] * sm.z[rr][i]; });
    } else if (p < kOW2) {
      const int m = p - kOB1;
      acc = sum_rows([&](int rr) { return sm.d1[rr][m]; });
    } else if (p < kOB2) {
      const int o = (p - kOW2) / kH, m = (p - kOW2) - o * kH;
      acc = sum_rows([&](int rr) { return sm.d2[rr][o] * sm.h1[rr][m]; });
    } else if (p < kOW3) {
      const int o = p - kOB2;
      acc = sum_rows([&](int rr) { return sm.d2[rr][o]; });
    } else if (p < kOB3) {
      const int o = (p - kOW3) / kH, m = (p - kOW3) - o * kH;
      acc = sum_rows([&](int rr) { return sm.ds[rr][o] * sm.h2[rr][m]; });
    } else {
      const int o = p - kOB3;
      acc = sum_rows([&](int rr) { return sm.ds[rr][o]; });
    }
    G[p] = old[u] + acc;
  }
}

// The Eq. 16 outlet of the workgroup's 64 rows: the node adjoints of the
// last three columns (the outlet column's stays in registers), then per row
// the network recomputed and its backward pass: the outlet node's adjoint
// lam_g of g3, g6, g7 is the adjoint of f_q(L-1) (left in the row's slot q
// with the features' adjoints) and, times sd_out, of the network's output;
// then the parameter-gradient sums of the rows.
template <typename T>
__global__ void __launch_bounds__(kBwdThreads) k_bwd_outlet_nn(const CtArgs<T> a, int k) {
  __shared__ BwdSmem<T> sm;
  __shared__ float sw[kNPNn];
  const int s = blockIdx.y;
  const int nt = a.nts[s];
  if (k >= nt) return;                           // uniform over the workgroup
  const int j = threadIdx.x;
  const int r = blockIdx.x * kRows + j;
  const CtState* st = a.st;
  const bool valid = r < a.ny;
  const int rl = valid ? r : a.ny - 1;
  T* LF = a.lamF[k & 1] + int64_t(s) * 9 * a.plane;
  T lf[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) lf[q] = T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (valid) {
      const int x = a.W - 1 - c;
      const int64_t n = int64_t(x) * a.ny + r;
      T l9[9];
      node_adjoint<T, kOutNn>(a, s, nt, k, x, r, n, l9);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        if (c == 0) lf[q] = l9[q];
        else LF[q * a.plane + n] = l9[q];
      }
    }
  }
  T fe[9];
  pull(state_at(a, s, k), a.plane, a.W, a.ny, a.W - 2, rl, fe);
  stage_weights(st, sw, kBwdThreads, kNPNn);
  if (valid) {
    const int64_t on = int64_t(a.W - 1) * a.ny + r;
    // the outlet node's known populations feed the streaming adjoint; its
    // unknowns have no source inside the strip
#pragma unroll
    for (int q = 0; q < 9; ++q) LF[q * a.plane + on] = (q == 3 || q == 6 || q == 7) ? T(0) : lf[q];
    T z[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) {
      z[i] = (fe[i] - T(st->mu[i])) / T(st->sd[i]);
      sm.z[j][i] = z[i];
    }
    // activations and tanh derivatives in LDS (the derivatives are scaled
    // into the pre-activation adjoints below)
#pragma unroll 1
    for (int o = 0; o < kH; ++o) {
      T acc = T(sw[kOB1 + o]);
#pragma unroll
      for (int i = 0; i < kIn; ++i) acc += T(sw[kOW1 + o * kIn + i]) * z[i];
      const T h = tanh_t(acc);
      sm.h1[j][o] = h;
      sm.d1[j][o] = T(1) - h * h;
    }
#pragma unroll 1
    for (int o = 0; o < kH; ++o) {
      T acc = T(sw[kOB2 + o]);
#pragma unroll 4
      for (int m = 0; m < kH; ++m) acc += T(sw[kOW2 + o * kH + m]) * sm.h1[j][m];
      const T h = tanh_t(acc);
      sm.h2[j][o] = h;
      sm.d2[j][o] = T(1) - h * h;
    }
    // s_i = o_i sd_out_i + mu_out_i, g_{3,6,7} = f_{3,6,7}(L-1) + s
    const T lo0 = lf[3] * T(st->sd_out[0]), lo1 = lf[6] * T(st->sd_out[1]),
            lo2 = lf[7] * T(st->sd_out[2]);
    sm.ds[j][0] = lo0;
    sm.ds[j][1] = lo1;
    sm.ds[j][2] = lo2;
#pragma unroll
    for (int o = 0; o < kH; ++o)
      sm.d2[j][o] *= T(sw[kOW3 + o]) * lo0 + T(sw[kOW3 + kH + o]) * lo1 +
                     T(sw[kOW3 + 2 * kH + o]) * lo2;
    T lz[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) lz[i] = T(0);
#pragma unroll 1
    for (int m = 0; m < kH; ++m) {
      T acc = T(0);
#pragma unroll
      for (int o = 0; o < kH; ++o) acc += T(sw[kOW2 + o * kH + m]) * sm.d2[j][o];
      const T d = acc * sm.d1[j][m];
      sm.d1[j][m] = d;
#pragma unroll
      for (int i = 0; i < kIn; ++i) lz[i] += T(sw[kOW1 + m * kIn + i]) * d;
    }
    T* P = a.madj[k & 1] + (int64_t(s) * a.ny + r) * kMadj;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      P[q] = lz[q] / T(st->sd[q]) + (q == 3 || q == 6 || q == 7 ? lf[q] : T(0));
  } else {
#pragma unroll
    for (int i = 0; i < kIn; ++i) sm.z[j][i] = T(0);
#pragma unroll
    for (int o = 0; o < kH; ++o) sm.h1[j][o] = sm.h2[j][o] = sm.d1[j][o] = sm.d2[j][o] = T(0);
    sm.ds[j][0] = sm.ds[j][1] = sm.ds[j][2] = T(0);
  }
  __syncthreads();
  double* G = a.gslot + (int64_t(s) * a.nrb + blockIdx.x) * kNPMax;
  constexpr int kPer = (kNPNn + kBwdThreads - 1) / kBwdThreads;
  double old[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int p = j + u * kBwdThreads;
    old[u] = p < kNPNn ? G[p] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int p = j + u * kBwdThreads;
    if (p >= kNPNn) break;
    T acc;
    if (p < kOB1) {
      const int m = p / kIn, i = p - m * kIn;
      acc = sum_rows([&](int rr) { return sm.d1[rr][m] * sm.z[rr][i]; });
    } else if (p < kOW2) {
      const int m = p - kOB1;
      acc = sum_rows([&](int rr) { return sm.d1[rr][m]; });
    } else if (p < kOB2) {
      const int o = (p - kOW2) / kH, m = (p - kOW2) - o * kH;
      acc = sum_rows([&](int rr) { return sm.d2[rr][o] * sm.h1[rr][m]; });
    } else if (p < kOW3) {
      const int o = p - kOB2;
      acc = sum_rows([&](int rr) { return sm.d2[rr][o]; });
    } else if (p < kOB3n) {
      const int o = (p - kOW3) / kH, m = (p - kOW3) - o * kH;
      acc = sum_rows([&](int rr) { return sm.ds[rr][o] * sm.h2[rr][m]; });
    } else {
      const int o = p - kOB3n;
      acc = sum_rows([&](int rr) { return sm.ds[rr][o]; });
    }
    G[p] = old[u] + acc;
  }
}

__global__ void k_zero(double* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Fixed-order FP64 sums in two stages.  k_gsum: workgroup (c, t) adds the
// gradient slots [c kSlotChunk, (c+1) kSlotChunk) of parameters
// 64 t .. 64 t + 63, four groups of kSlotChunk/4 consecutive slots combined
// in order; k_lsum: each workgroup adds kLossChunk consecutive loss slots.
constexpr int kSlotChunk = 64;
constexpr int kLossChunk = 4 * kNodes;

__global__ void __launch_bounds__(kNodes) k_gsum(const double* gslot, int64_t nslots,
                                                double* gpart, int np) {
  __shared__ double sh[4][64];
  const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int p = blockIdx.y * 64 + l;
  const int64_t i0 = int64_t(blockIdx.x) * kSlotChunk + g * (kSlotChunk / 4);
  double acc = 0.0;
  if (p < np) {
#pragma unroll 4
    for (int j = 0; j < kSlotChunk / 4; ++j) {
      const int64_t i = i0 + j;
      if (i < nslots) acc += gslot[i * kNPMax + p];
    }
  }
  sh[g][l] = acc;
  __syncthreads();
  if (g == 0 && p < np)
    gpart[int64_t(blockIdx.x) * kNPMax + p] = (sh[0][l] + sh[1][l]) + (sh[2][l] + sh[3][l]);
}

__global__ void __launch_bounds__(kNodes) k_lsum(const double* lslot, int64_t nl, double* lpart) {
  __shared__ double sh[kNodes / 64];
  const int64_t i0 = int64_t(blockIdx.x) * kLossChunk + 4 * threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (i0 + j < nl) acc += lslot[i0 + j];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) lpart[blockIdx.x] = t;
}

// Second stage (chunk order) and Adam with bias correction when `update`.
__global__ void __launch_bounds__(kNodes) k_update(CtState* st, const double* gpart, int ngc,
                                                  const double* lpart, int nlc, int update,
                                                  double lr, double b1, double b2, double eps,
                                                  double bc1, double bc2, int np) {
  const int p = blockIdx.x * kNodes + threadIdx.x;
  if (p == 0) {
    double t = 0.0;
    for (int i = 0; i < nlc; ++i) t += lpart[i];
    st->loss = t;
  }
  if (p >= np) return;
  double g = 0.0;
  for (int i = 0; i < ngc; ++i) g += gpart[int64_t(i) * kNPMax + p];
  st->grad[p] = g;
  if (update) {
    const double m = b1 * st->m[p] + (1.0 - b1) * g;
    const double v = b2 * st->v[p] + (1.0 - b2) * g * g;
    st->m[p] = m;
    st->v[p] = v;
    st->w[p] = float(double(st->w[p]) - lr * (m / bc1) / (sqrt(v / bc2) + eps));
  }
}

// ---- host side ---------------------------------------------------------------------------
size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct CtLayout {
  size_t st, traj, outs, dts, lamF, lamP, madj, ref, nts, seg_omega, seg_k1c, gslot, lslot,
      gpart, lpart, total;
  int W, nrb, nlb, ngc, nlc;      // gradient / loss chunks of the first-stage sums
  int64_t plane;
};

size_t elem(int precision) { return precision == LBM_FP64 ? 8 : 4; }

CtLayout ct_layout(const lbm_cbc_train_params& p) {
  CtLayout L;
  L.W = 2 * p.n_max + 3;
  L.plane = int64_t(p.ny) * L.W;
  L.nrb = (p.ny + kRows - 1) / kRows;
  L.nlb = int((L.plane + kNodes - 1) / kNodes);
  L.ngc = int((int64_t(p.n_seg) * L.nrb + kSlotChunk - 1) / kSlotChunk);
  L.nlc = int((int64_t(p.n_seg) * L.nlb + kLossChunk - 1) / kLossChunk);
  const size_t e = elem(p.precision), ns = size_t(p.n_seg), ny = size_t(p.ny);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.st = take(sizeof(CtState));
  L.traj = take(ns * (p.n_max + 1) * 9 * size_t(L.plane) * e);
  L.outs = take(ns * p.n_max * ny * 3 * e);
  L.dts = take(ns * (p.n_max + 1) * ny * 3 * e);
  L.lamF = take(2 * ns * 9 * size_t(L.plane) * e);
  L.lamP = take(ns * ny * 3 * e);
  L.madj = take(2 * ns * ny * kMadj * e);
  L.ref = take(ns * 3 * ny * p.n_max * e);
  L.nts = take(ns * sizeof(int));
  L.gslot = take(ns * L.nrb * kNPMax * sizeof(double));
  L.lslot = take(ns * L.nlb * sizeof(double));
  L.gpart = take(size_t(L.ngc) * kNPMax * sizeof(double));
  L.lpart = take(size_t(L.nlc) * sizeof(double));
  L.seg_omega = take(ns * sizeof(double));
  L.seg_k1c = take(ns * sizeof(double));
  L.total = o;
  return L;
}

lbm_status check_params(const lbm_cbc_train_params* p) {
  if (!p) return set_error(LBM_EINVAL, "params is NULL");
  if (p->ny < 3) return set_error(LBM_EINVAL, "ny must be >= 3");
  if (p->n_max < 1 || p->n_max > kMaxSteps) return set_error(LBM_EINVAL, "n_max must be in 1..%d", kMaxSteps);
  if (p->n_seg < 1 || p->n_seg > 65535) return set_error(LBM_EINVAL, "n_seg must be in 1..65535");
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32_OFFSET)
    return set_error(LBM_EINVAL, "precision must be LBM_FP64 or LBM_FP32_OFFSET");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return set_error(LBM_EINVAL, "tau must be > 1/2");
  if (!(p->mach >= 0.0 && p->mach < 1.0)) return set_error(LBM_EINVAL, "mach must be in [0, 1)");
  if (!(p->length > 0.0) || !std::isfinite(p->length)) return set_error(LBM_EINVAL, "length must be > 0");
  if (!(p->rho_inf > 0.0) || !std::isfinite(p->rho_inf)) return set_error(LBM_EINVAL, "rho_inf must be > 0");
  if (!(p->lr > 0.0) || !(p->beta1 >= 0.0 && p->beta1 < 1.0) || !(p->beta2 >= 0.0 && p->beta2 < 1.0) ||
      !(p->eps > 0.0))
    return set_error(LBM_EINVAL, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
  if (int64_t(p->ny) * (2 * p->n_max + 3) >= (int64_t(1) << 31) / 9)
    return set_error(LBM_EINVAL, "strip too large");
  return LBM_OK;
}

#define CT_TRY(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return set_error(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_cbc_trainer {
  lbm_cbc_train_params p;
  hipStream_t stream;
  hipStream_t side = nullptr;                  // the outlet kernels' stream
  hipEvent_t ev_node = nullptr, ev_side = nullptr;
  CtLayout L;
  char* base;
  CtState* st;
  std::vector<int> nts;
  bool has_data = false, has_net = false;
  int kind = kOutCbc;                          // the outlet the network set drives
  int64_t adam_t = 0;

  int np() const { return kind == kOutNn ? kNPNn : kNP; }

  template <typename T>
  CtArgs<T> args() const {
    CtArgs<T> a;
    a.traj = reinterpret_cast<T*>(base + L.traj);
    a.outs = reinterpret_cast<T*>(base + L.outs);
    a.dts = reinterpret_cast<T*>(base + L.dts);
    a.lamF[0] = reinterpret_cast<T*>(base + L.lamF);
    a.lamF[1] = a.lamF[0] + size_t(p.n_seg) * 9 * size_t(L.plane);
    a.lamP = reinterpret_cast<T*>(base + L.lamP);
    a.madj[0] = reinterpret_cast<T*>(base + L.madj);
    a.madj[1] = a.madj[0] + size_t(p.n_seg) * size_t(p.ny) * kMadj;
    a.ref = reinterpret_cast<const T*>(base + L.ref);
    a.nts = reinterpret_cast<const int*>(base + L.nts);
    a.gslot = reinterpret_cast<double*>(base + L.gslot);
    a.lslot = reinterpret_cast<double*>(base + L.lslot);
    a.st = st;
    a.ny = p.ny;
    a.W = L.W;
    a.n_max = p.n_max;
    a.nrb = L.nrb;
    a.nlb = L.nlb;
    a.nlb_fwd = int((L.plane - p.ny + kNodes - 1) / kNodes);
    a.nlb_bwd = int((L.plane - 3 * int64_t(p.ny) + kNodes - 1) / kNodes);
    a.nrb_fwd = (p.ny + kNodes - 1) / kNodes;
    a.n_seg = p.n_seg;
    a.plane = L.plane;
    a.seg_omega = reinterpret_cast<const double*>(base + L.seg_omega);
    a.seg_k1c = reinterpret_cast<const double*>(base + L.seg_k1c);
    a.seg_scale = 1.0 / double(p.n_seg);
    return a;
  }

  // One step on both streams: each first waits for the other's previous
  // step (a wait takes the event's latest record at the time of the call).
  hipError_t join_step() {
    const hipError_t e = hipStreamWaitEvent(stream, ev_side, 0);
    return e != hipSuccess ? e : hipStreamWaitEvent(side, ev_node, 0);
  }

  template <typename T, int OK>
  lbm_status run_t(bool update) {
    const CtArgs<T> a = args<T>();
    const dim3 grow(L.nrb, p.n_seg), gnode(L.nlb, p.n_seg);
    const dim3 gbwd(a.nlb_bwd, p.n_seg);
    const unsigned gf = unsigned(p.n_seg) * unsigned(a.nrb_fwd + a.nlb_fwd);
    for (int k = 0; k < p.n_max; ++k)
      hipLaunchKernelGGL((k_fwd<T, OK>), dim3(gf), dim3(kNodes), 0, stream, a, k);
    const int64_t ng = int64_t(p.n_seg) * L.nrb * kNPMax;
    hipLaunchKernelGGL(k_zero, dim3(unsigned((ng + kNodes - 1) / kNodes)), dim3(kNodes), 0, stream,
                       a.gslot, ng);
    hipLaunchKernelGGL(k_seed<T>, gnode, dim3(kNodes), 0, stream, a);
    CT_TRY(hipEventRecord(ev_node, stream));
    CT_TRY(hipEventRecord(ev_side, side));
    for (int k = p.n_max - 1; k >= 0; --k) {
      CT_TRY(join_step());
      if constexpr (OK == kOutNn)
        hipLaunchKernelGGL(k_bwd_outlet_nn<T>, grow, dim3(kBwdThreads), 0, side, a, k);
      else
        hipLaunchKernelGGL(k_bwd_outlet<T>, grow, dim3(kBwdThreads), 0, side, a, k);
      CT_TRY(hipEventRecord(ev_side, side));
      hipLaunchKernelGGL((k_bwd<T, OK>), gbwd, dim3(kNodes), 0, stream, a, k);
      CT_TRY(hipEventRecord(ev_node, stream));
    }
    CT_TRY(hipStreamWaitEvent(stream, ev_side, 0));
    double bc1 = 1.0, bc2 = 1.0;
    if (update) {
      bc1 = 1.0 - std::pow(p.beta1, double(adam_t));
      bc2 = 1.0 - std::pow(p.beta2, double(adam_t));
    }
    double* gpart = reinterpret_cast<double*>(base + L.gpart);
    double* lpart = reinterpret_cast<double*>(base + L.lpart);
    hipLaunchKernelGGL(k_gsum, dim3(L.ngc, (np() + 63) / 64), dim3(kNodes), 0, stream, a.gslot,
                       int64_t(p.n_seg) * L.nrb, gpart, np());
    hipLaunchKernelGGL(k_lsum, dim3(L.nlc), dim3(kNodes), 0, stream, a.lslot,
                       int64_t(p.n_seg) * L.nlb, lpart);
    hipLaunchKernelGGL(k_update, dim3((np() + kNodes - 1) / kNodes), dim3(kNodes), 0, stream, st,
                       gpart, L.ngc, lpart, L.nlc,
                       update ? 1 : 0, p.lr, p.beta1, p.beta2, p.eps, bc1, bc2, np());
    CT_TRY(hipGetLastError());
    return LBM_OK;
  }

  lbm_status run(bool update) {
    if (!has_data || !has_net) return set_error(LBM_ESTATE, "segments and network must be set first");
    // the second stream and the events: made on the first run, on the
    // device current then
    if (!ev_node) CT_TRY(hipEventCreateWithFlags(&ev_node, kEventFlags));
    if (!ev_side) CT_TRY(hipEventCreateWithFlags(&ev_side, kEventFlags));
    if (!side) CT_TRY(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    if (kind == kOutNn)
      return p.precision == LBM_FP64 ? run_t<double, kOutNn>(update) : run_t<float, kOutNn>(update);
    return p.precision == LBM_FP64 ? run_t<double, kOutCbc>(update) : run_t<float, kOutCbc>(update);
  }
};

// Per-segment relaxation and kappa_1 coefficient (host arrays of n_seg, or
// NULL for the trainer's own tau / mach), copied to the device.
lbm_status set_seg_params(lbm_cbc_trainer* t, const double* tau, const double* mach) {
  const lbm_cbc_train_params& p = t->p;
  const double cs = 0.57735026918962576451;
  std::vector<double> om(size_t(p.n_seg)), k1(size_t(p.n_seg));
  for (int s = 0; s < p.n_seg; ++s) {
    const double ta = tau ? tau[s] : p.tau, ma = mach ? mach[s] : p.mach;
    if (!(ta > 0.5) || !std::isfinite(ta)) return set_error(LBM_EINVAL, "tau[%d] must be > 1/2", s);
    if (!(ma >= 0.0 && ma < 1.0)) return set_error(LBM_EINVAL, "mach[%d] must be in [0, 1)", s);
    om[size_t(s)] = 1.0 / ta;
    k1[size_t(s)] = (1.0 - ma * ma) * cs / p.length;
  }
  CT_TRY(hipMemcpyAsync(t->base + t->L.seg_omega, om.data(), om.size() * 8, hipMemcpyHostToDevice,
                        t->stream));
  CT_TRY(hipMemcpyAsync(t->base + t->L.seg_k1c, k1.data(), k1.size() * 8, hipMemcpyHostToDevice,
                        t->stream));
  CT_TRY(hipStreamSynchronize(t->stream));
  return LBM_OK;
}

extern "C" {

size_t lbm_cbc_train_workspace_bytes(const lbm_cbc_train_params* p) {
  if (check_params(p)) return 0;
  return ct_layout(*p).total;
}

lbm_status lbm_cbc_train_create(const lbm_cbc_train_params* p, void* ws, size_t bytes,
                                lbm_cbc_trainer** out) {
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status s = check_params(p);
  if (s) return s;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256)
    return set_error(LBM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  const CtLayout L = ct_layout(*p);
  if (bytes < L.total) return set_error(LBM_ENOSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);
  lbm_cbc_trainer* t = new lbm_cbc_trainer();
  t->p = *p;
  t->stream = static_cast<hipStream_t>(p->stream);
  t->L = L;
  t->base = static_cast<char*>(ws);
  t->st = reinterpret_cast<CtState*>(t->base + L.st);
  *out = t;
  return LBM_OK;
}

lbm_status lbm_cbc_train_destroy(lbm_cbc_trainer* t) {
  if (!t) return LBM_OK;
  (void)hipStreamSynchronize(t->stream);
  if (t->side) {
    (void)hipStreamSynchronize(t->side);
    (void)hipStreamDestroy(t->side);
  }
  if (t->ev_node) (void)hipEventDestroy(t->ev_node);
  if (t->ev_side) (void)hipEventDestroy(t->ev_side);
  delete t;
  return LBM_OK;
}

lbm_status lbm_cbc_train_set_segments(lbm_cbc_trainer* t, const double* a0, const double* ref,
                                      const int32_t* n_t) {
  if (!t || !a0 || !ref || !n_t) return set_error(LBM_EINVAL, "NULL argument");
  const lbm_cbc_train_params& p = t->p;
  const CtLayout& L = t->L;
  for (int s = 0; s < p.n_seg; ++s)
    if (n_t[s] < 1 || n_t[s] > p.n_max) return set_error(LBM_EINVAL, "n_t[%d] = %d outside 1..%d", s, n_t[s], p.n_max);
  const size_t seg_vals = size_t(9) * size_t(L.plane);
  const size_t ref_vals = size_t(3) * size_t(p.ny) * size_t(p.n_max);
  for (size_t i = 0; i < seg_vals * size_t(p.n_seg); ++i)
    if (!std::isfinite(a0[i])) return set_error(LBM_EINVAL, "a0 holds a non-finite value");
  const bool f64 = p.precision == LBM_FP64;
  const size_t e = elem(p.precision);
  std::vector<char> h(seg_vals * size_t(p.n_seg) * e);
  std::vector<char> hr(ref_vals * size_t(p.n_seg) * e);
  // caller layout [seg][9][ny][W] -> device planes [seg][9][W][ny], offsets
  const size_t W = size_t(L.W), ny = size_t(p.ny);
  for (size_t sq = 0; sq < size_t(p.n_seg) * 9; ++sq) {
    const int q = int(sq % 9);
    const double wq = q == 0 ? 4.0 / 9.0 : (q <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    const double* src = a0 + sq * size_t(L.plane);
    for (size_t y = 0; y < ny; ++y)
      for (size_t x = 0; x < W; ++x) {
        const double g = src[y * W + x] - wq;
        const size_t d = sq * size_t(L.plane) + x * ny + y;
        if (f64) reinterpret_cast<double*>(h.data())[d] = g;
        else reinterpret_cast<float*>(h.data())[d] = float(g);
      }
  }
  for (size_t i = 0; i < ref_vals * size_t(p.n_seg); ++i) {
    const int c = int((i / (size_t(p.ny) * size_t(p.n_max))) % 3);
    const double v = c == 0 ? ref[i] - 1.0 : ref[i];      // density as rho - 1
    if (f64) reinterpret_cast<double*>(hr.data())[i] = v;
    else reinterpret_cast<float*>(hr.data())[i] = float(v);
  }
  CT_TRY(hipMemcpy2DAsync(t->base + L.traj, size_t(p.n_max + 1) * seg_vals * e, h.data(), seg_vals * e,
                          seg_vals * e, size_t(p.n_seg), hipMemcpyHostToDevice, t->stream));
  CT_TRY(hipMemcpyAsync(t->base + L.ref, hr.data(), hr.size(), hipMemcpyHostToDevice, t->stream));
  t->nts.assign(n_t, n_t + p.n_seg);
  {
    lbm_status st = set_seg_params(t, nullptr, nullptr);
    if (st) return st;
  }
  CT_TRY(hipMemcpyAsync(t->base + L.nts, t->nts.data(), t->nts.size() * sizeof(int),
                        hipMemcpyHostToDevice, t->stream));
  CT_TRY(hipMemsetAsync(t->base + L.dts, 0, size_t(p.n_seg) * (p.n_max + 1) * p.ny * 3 * e, t->stream));
  CT_TRY(hipStreamSynchronize(t->stream));
  t->has_data = true;
  return LBM_OK;
}

lbm_status lbm_cbc_train_set_segment_params(lbm_cbc_trainer* t, const double* tau,
                                            const double* mach) {
  if (!t) return set_error(LBM_EINVAL, "NULL trainer");
  if (!t->has_data) return set_error(LBM_ESTATE, "set the segments first");
  return set_seg_params(t, tau, mach);
}

lbm_status lbm_cbc_train_set_net(lbm_cbc_trainer* t, const lbm_cbc_net* n) {
  if (!t || !n || !n->w1 || !n->b1 || !n->w2 || !n->b2 || !n->w3 || !n->b3 || !n->mu_in || !n->sd_in)
    return set_error(LBM_EINVAL, "NULL argument");
  std::vector<char> buf(sizeof(CtState), 0);
  CtState* h = reinterpret_cast<CtState*>(buf.data());
  memcpy(h->w + kOW1, n->w1, kH * kIn * 4);
  memcpy(h->w + kOB1, n->b1, kH * 4);
  memcpy(h->w + kOW2, n->w2, kH * kH * 4);
  memcpy(h->w + kOB2, n->b2, kH * 4);
  memcpy(h->w + kOW3, n->w3, 2 * kH * 4);
  memcpy(h->w + kOB3, n->b3, 2 * 4);
  for (int i = 0; i < kNP; ++i)
    if (!std::isfinite(h->w[i])) return set_error(LBM_EINVAL, "non-finite weight %d", i);
  for (int i = 0; i < kIn; ++i) {
    if (!std::isfinite(n->mu_in[i]) || !(n->sd_in[i] > 0.0f) || !std::isfinite(n->sd_in[i]))
      return set_error(LBM_EINVAL, "mu_in must be finite and sd_in > 0");
    h->mu[i] = n->mu_in[i];
    h->sd[i] = n->sd_in[i];
  }
  const double maps[5] = {n->leaky_slope, n->sigma_scale, n->sigma_shift, n->kappa_scale, n->kappa_shift};
  for (double v : maps)
    if (!std::isfinite(v)) return set_error(LBM_EINVAL, "non-finite slope or output map");
  h->leaky = n->leaky_slope;
  h->sig_scale = n->sigma_scale;
  h->sig_shift = n->sigma_shift;
  h->kap_scale = n->kappa_scale;
  h->kap_shift = n->kappa_shift;
  h->rho_inf_m1 = t->p.rho_inf - 1.0;
  CT_TRY(hipMemcpyAsync(t->st, h, sizeof(CtState), hipMemcpyHostToDevice, t->stream));
  CT_TRY(hipStreamSynchronize(t->stream));
  t->adam_t = 0;
  t->kind = kOutCbc;
  t->has_net = true;
  return LBM_OK;
}

lbm_status lbm_cbc_train_set_nn(lbm_cbc_trainer* t, const lbm_nn9_net* n) {
  if (!t || !n) return set_error(LBM_EINVAL, "NULL argument");
  std::vector<char> buf(sizeof(CtState), 0);
  CtState* h = reinterpret_cast<CtState*>(buf.data());
  memcpy(h->w + kOW1, n->w1, kH * kIn * 4);
  memcpy(h->w + kOB1, n->b1, kH * 4);
  memcpy(h->w + kOW2, n->w2, kH * kH * 4);
  memcpy(h->w + kOB2, n->b2, kH * 4);
  memcpy(h->w + kOW3, n->w3, 3 * kH * 4);
  memcpy(h->w + kOB3n, n->b3, 3 * 4);
  for (int i = 0; i < kNPNn; ++i)
    if (!std::isfinite(h->w[i])) return set_error(LBM_EINVAL, "non-finite weight %d", i);
  for (int i = 0; i < kIn; ++i) {
    if (!std::isfinite(n->mu_in[i]) || !(n->sd_in[i] > 0.0f) || !std::isfinite(n->sd_in[i]))
      return set_error(LBM_EINVAL, "mu_in must be finite and sd_in > 0");
    h->mu[i] = n->mu_in[i];
    h->sd[i] = n->sd_in[i];
  }
  for (int i = 0; i < 3; ++i) {
    if (!std::isfinite(n->mu_out[i]) || !(n->sd_out[i] > 0.0f) || !std::isfinite(n->sd_out[i]))
      return set_error(LBM_EINVAL, "mu_out must be finite and sd_out > 0");
    h->mu_out[i] = n->mu_out[i];
    h->sd_out[i] = n->sd_out[i];
  }
  CT_TRY(hipMemcpyAsync(t->st, h, sizeof(CtState), hipMemcpyHostToDevice, t->stream));
  CT_TRY(hipStreamSynchronize(t->stream));
  t->adam_t = 0;
  t->kind = kOutNn;
  t->has_net = true;
  return LBM_OK;
}

lbm_status lbm_cbc_train_gradient(lbm_cbc_trainer* t, double* loss, double* grad) {
  if (!t) return set_error(LBM_EINVAL, "NULL trainer");
  lbm_status s = t->run(false);
  if (s) return s;
  CT_TRY(hipStreamSynchronize(t->stream));
  if (loss) CT_TRY(hipMemcpy(loss, &t->st->loss, sizeof(double), hipMemcpyDeviceToHost));
  if (grad) CT_TRY(hipMemcpy(grad, t->st->grad, t->np() * sizeof(double), hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_cbc_train_step(lbm_cbc_trainer* t, int64_t nsteps) {
  if (!t) return set_error(LBM_EINVAL, "NULL trainer");
  if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps < 0");
  for (int64_t i = 0; i < nsteps; ++i) {
    ++t->adam_t;
    lbm_status s = t->run(true);
    if (s) return s;
  }
  return LBM_OK;
}

lbm_status lbm_cbc_train_loss(lbm_cbc_trainer* t, double* loss) {
  if (!t || !loss) return set_error(LBM_EINVAL, "NULL argument");
  CT_TRY(hipStreamSynchronize(t->stream));
  CT_TRY(hipMemcpy(loss, &t->st->loss, sizeof(double), hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_cbc_train_get_weights(lbm_cbc_trainer* t, float* theta) {
  if (!t || !theta) return set_error(LBM_EINVAL, "NULL argument");
  CT_TRY(hipStreamSynchronize(t->stream));
  CT_TRY(hipMemcpy(theta, t->st->w, t->np() * sizeof(float), hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_cbc_train_final_state(lbm_cbc_trainer* t, int32_t seg, double* host) {
  if (!t || !host) return set_error(LBM_EINVAL, "NULL argument");
  if (!t->has_data) return set_error(LBM_ESTATE, "no segments set");
  if (seg < 0 || seg >= t->p.n_seg) return set_error(LBM_EINVAL, "seg outside 0..n_seg-1");
  const CtLayout& L = t->L;
  const size_t vals = size_t(9) * size_t(L.plane), e = elem(t->p.precision);
  const size_t off = L.traj + (size_t(seg) * (t->p.n_max + 1) + t->nts[seg]) * vals * e;
  std::vector<char> h(vals * e);
  CT_TRY(hipStreamSynchronize(t->stream));
  CT_TRY(hipMemcpy(h.data(), t->base + off, h.size(), hipMemcpyDeviceToHost));
  const size_t W = size_t(L.W), ny = size_t(t->p.ny);
  for (size_t q = 0; q < 9; ++q) {
    const double w = q == 0 ? 4.0 / 9.0 : (q <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    for (size_t y = 0; y < ny; ++y)
      for (size_t x = 0; x < W; ++x) {
        const size_t d = q * size_t(L.plane) + x * ny + y;
        const double g = e == 8 ? reinterpret_cast<double*>(h.data())[d]
                                : double(reinterpret_cast<float*>(h.data())[d]);
        host[q * size_t(L.plane) + y * W + x] = g + w;
      }
  }
  return LBM_OK;
}

}  // extern "C"
