// D3Q19 step on gfx950 (C ABI of include/lbm3d.h): the method's step carried
// to three dimensions.
//
// One launch per step, k3_step: one node per thread, 256 nodes along x per
// workgroup, workgroups remapped so that each XCD takes a contiguous range
// of (y, z) rows (the pulls from rows y +- 1 and z +- 1 then meet in the same
// L2).  Per node: pull streaming of the 19 populations (a source outside the
// x-range is an unknown of the inlet or outlet face, a source outside y or z
// bounces back off a wall or wraps round, a solid source -- a bit of the
// node's link word -- bounces back half-way and adds the momentum exchange
// to the force), the Zou & He face at x = 0 or x = nx-1, BGK collision in
// offset form g = f - w, non-temporal stores.  Each workgroup leaves one FP64
// partial of (F_x, F_y, F_z, sum rho - 1) in a ring of kRing step slots;
// k3_reduce adds them in a fixed order, one workgroup per step, for up to
// kRing steps per launch (and before any read of the forces), and appends
// the forces to the history.
//
// HBM traffic per node and step (FP32): 19 loads + 19 stores + the link
// word = 156 B (152 B algorithmic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lbm3d.h"
#include "lbm_internal.hpp"

namespace lbm {
namespace {

// Velocities in the numbering of lbm3d.h.
__host__ __device__ constexpr int c3(int q, int a) {
  constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},
                            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                            {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
                            {0, 1, 1},  {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
  return t[q][a];
}
__host__ __device__ constexpr int opp3(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
template <typename T>
__host__ __device__ constexpr T w3(int q) {
  return q == 0 ? T(1) / T(3) : (q <= 6 ? T(1) / T(18) : T(1) / T(36));
}
static_assert(opp3(7) == 8 && opp3(8) == 7 && c3(7, 0) == -c3(8, 0) && c3(17, 2) == -c3(18, 2),
              "opposites");

constexpr uint32_t kSolid3 = 1u << 24;    // link word: the node itself is solid
constexpr int kB3 = 256;                  // nodes per row of a workgroup (along x)
// (y, z) rows per workgroup: two or four rows (larger contiguous pieces of
// each population plane per workgroup) measured 1.7 % and 4.4 % slower
constexpr int kR3 = 1;
constexpr int kT3 = kB3 * kR3;             // threads per workgroup

struct Step3 {
  const void* A;
  void* B;
  const uint32_t* links;
  const uint8_t* rowf;   // [nz][ny]: 1 where the row holds a solid node or a body link
  double* part;          // [nblocks][4]
  int nx, ny, nz, pitch, ntx, nblocks;
  int chunk;             // workgroups per chunk dealt to an XCD
  int64_t plane;         // nz * ny * pitch
  int xper, yper, zper;
  double omega, u_in, one_minus_rho_out;
};

__device__ __forceinline__ int xcd_range(int bid, int n) {
  const int q = n >> 3, r = n & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

// Chunks of S workgroups dealt to the XCDs in turn (XCD x takes chunks x,
// x + 8, ...), the tail after the last full round by xcd_range: the eight
// XCDs then work on nearby rows at any time.  With S the rows of ~512 KiB of
// a plane: 118.4 vs 121.6 us per step at 256 x 128 x 128 against one range
// per XCD, and 5-7 % at 120 and 136 rows, where the ranges' spacing loads
// the HBM channels unevenly.
__device__ __forceinline__ int xcd_chunks(int bid, int n, int S) {
  const int full = n / (8 * S) * (8 * S);
  if (bid >= full) return full + xcd_range(bid - full, n - full);
  const int x = bid & 7, k = bid >> 3;
  return ((k / S) * 8 + x) * S + k % S;
}

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Zou & He faces in offset form.  The weights of the populations with
// c_x = 0 plus twice those entering from the outside sum to 1, so
// rho (1 - u) = 1 + d0 + 2 d_- at the inlet and rho u = d0 + 2 d_+ + 1 - rho_out
// at the outlet; the unknowns are the opposite populations plus
// 6 w_i rho c_i.u (rho u / 3 on the axis, rho u / 6 on the edges), then the
// edge unknowns with a transverse component take -c_t N_t with N_t half the
// transverse momentum the node carries (the prescribed one is zero).
template <typename T>
__device__ __forceinline__ void face_transverse(T g[19], int sgn) {
  const T ny = T(0.5) * ((g[3] - g[4]) + (g[7] - g[8]) - (g[9] - g[10]) + (g[15] - g[16]) +
                         (g[17] - g[18]));
  const T nz = T(0.5) * ((g[5] - g[6]) + (g[11] - g[12]) - (g[13] - g[14]) + (g[15] - g[16]) -
                         (g[17] - g[18]));
  if (sgn > 0) {          // unknowns 7 (c_y +1), 9 (c_y -1), 11 (c_z +1), 13 (c_z -1)
    g[7] -= ny;
    g[9] += ny;
    g[11] -= nz;
    g[13] += nz;
  } else {                // unknowns 8 (c_y -1), 10 (c_y +1), 12 (c_z -1), 14 (c_z +1)
    g[8] += ny;
    g[10] -= ny;
    g[12] += nz;
    g[14] -= nz;
  }
}

template <typename T>
__device__ __forceinline__ T face_d0(const T g[19]) {
  return (g[0] + g[3] + g[4]) + (g[5] + g[6]) + ((g[15] + g[16]) + (g[17] + g[18]));
}

template <typename T>
__device__ __forceinline__ void inlet3(T g[19], T u) {
  const T dm = g[2] + ((g[8] + g[10]) + (g[12] + g[14]));
  const T drho = (face_d0(g) + T(2) * dm + u) / (T(1) - u);
  const T ru = (T(1) + drho) * u;
  g[1] = g[2] + ru * T(1.0 / 3.0);
  g[7] = g[8] + ru * T(1.0 / 6.0);
  g[9] = g[10] + ru * T(1.0 / 6.0);
  g[11] = g[12] + ru * T(1.0 / 6.0);
  g[13] = g[14] + ru * T(1.0 / 6.0);
  face_transverse(g, 1);
}

template <typename T>
__device__ __forceinline__ void outlet3(T g[19], T one_minus_rho_out) {
  const T dp = g[1] + ((g[7] + g[9]) + (g[11] + g[13]));
  const T ru = face_d0(g) + T(2) * dp + one_minus_rho_out;
  g[2] = g[1] - ru * T(1.0 / 3.0);
  g[8] = g[7] - ru * T(1.0 / 6.0);
  g[10] = g[9] - ru * T(1.0 / 6.0);
  g[12] = g[11] - ru * T(1.0 / 6.0);
  g[14] = g[13] - ru * T(1.0 / 6.0);
  face_transverse(g, -1);
}

// BGK (Eq. 2) in offset form: g^eq_i = w_i (drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)).
template <typename T>
__device__ __forceinline__ T bgk3(T g[19], T omega) {
  T drho = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    drho += g[q];
    if (c3(q, 0)) jx += T(c3(q, 0)) * g[q];
    if (c3(q, 1)) jy += T(c3(q, 1)) * g[q];
    if (c3(q, 2)) jz += T(c3(q, 2)) * g[q];
  }
  const T rho = T(1) + drho, inv = T(1) / rho;
  const T ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const T usq = T(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const T cu = T(c3(q, 0)) * ux + T(c3(q, 1)) * uy + T(c3(q, 2)) * uz;
    const T geq = w3<T>(q) * (drho + rho * (T(3) * cu + T(4.5) * cu * cu - usq));
    g[q] = g[q] - omega * (g[q] - geq);
  }
  return drho;
}

template <typename T>
__global__ void __launch_bounds__(kT3) k3_step(const Step3 L) {
  __shared__ double sh[kT3 / 64][4];
  const int v = xcd_chunks(int(blockIdx.x), L.nblocks, L.chunk);
  const int tx = v % L.ntx;
  const int row = (v / L.ntx) * kR3 + int(threadIdx.x) / kB3;
  const int y = row % L.ny, z = row / L.ny;
  const int x = tx * kB3 + int(threadIdx.x) % kB3;
  T fx = T(0), fy = T(0), fz = T(0), dm = T(0);
  if (x < L.nx && z < L.nz) {
    const int64_t idx = (int64_t(z) * L.ny + y) * L.pitch + x;
    // rows far from the body hold no link word worth reading (4 of the
    // 156 bytes per node)
    const uint32_t lk = L.rowf[row] ? L.links[idx] : 0u;
    if (!(lk & kSolid3)) {
      const T* __restrict__ A = static_cast<const T*>(L.A);
      T g[19];
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        int sx = x - c3(q, 0), sy = y - c3(q, 1), sz = z - c3(q, 2);
        bool xout = false, bb = (lk >> q) & 1u;
        if (sx < 0 || sx >= L.nx) {
          if (L.xper) sx = sx < 0 ? sx + L.nx : sx - L.nx;
          else xout = true;
        }
        if (sy < 0 || sy >= L.ny) {
          if (L.yper) sy = sy < 0 ? sy + L.ny : sy - L.ny;
          else bb = true;
        }
        if (sz < 0 || sz >= L.nz) {
          if (L.zper) sz = sz < 0 ? sz + L.nz : sz - L.nz;
          else bb = true;
        }
        if (xout) {
          g[q] = T(0);                                        // unknown of a face
        } else if (bb) {
          g[q] = __builtin_nontemporal_load(A + opp3(q) * L.plane + idx);
          if ((lk >> q) & 1u) {                               // a body link
            const T m = T(-2) * (g[q] + w3<T>(q));
            fx += m * T(c3(q, 0));
            fy += m * T(c3(q, 1));
            fz += m * T(c3(q, 2));
          }
        } else {
          g[q] = __builtin_nontemporal_load(A + q * L.plane + (int64_t(sz) * L.ny + sy) * L.pitch + sx);
        }
      }
      if (!L.xper) {
        if (x == 0) inlet3(g, T(L.u_in));
        else if (x == L.nx - 1) outlet3(g, T(L.one_minus_rho_out));
      }
      dm = bgk3(g, T(L.omega));
      T* __restrict__ B = static_cast<T*>(L.B);
#pragma unroll
      for (int q = 0; q < 19; ++q) __builtin_nontemporal_store(g[q], B + q * L.plane + idx);
    }
  }
  // workgroup partial in FP64, waves combined in order
  const double p[4] = {wsum(double(fx)), wsum(double(fy)), wsum(double(fz)), wsum(double(dm))};
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 4; ++c) sh[w][c] = p[c];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kT3 / 64; i += 4) t += (sh[i][c] + sh[i + 1][c]) + (sh[i + 2][c] + sh[i + 3][c]);
    L.part[int64_t(v) * 4 + c] = t;
  }
}

// Fixed-order sum of the workgroup partials of steps t0 .. t0 + gridDim.x - 1
// (workgroup j takes step t0 + j, ring slot (t0 + j) % kRing): thread t adds
// partials t, t + 1024, ... (coalesced reads), then a tree; appends the force
// to the history, the last step also to `last`, and records a non-finite sum.
constexpr int kRed3 = 1024;
constexpr int kRing = 16;

__global__ void __launch_bounds__(kRed3) k3_reduce(const double* ring, int nblocks, double* last,
                                                   double* hist, int64_t t0, int64_t cap) {
  __shared__ double sh[4][kRed3];
  const int64_t t = t0 + blockIdx.x;
  const double* part = ring + (t % kRing) * int64_t(nblocks) * 4;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kRed3) {
    const double4 v = reinterpret_cast<const double4*>(part)[b];
    s[0] += v.x;
    s[1] += v.y;
    s[2] += v.z;
    s[3] += v.w;
  }
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int o = kRed3 / 2; o >= 1; o >>= 1) {
    if (int(threadIdx.x) < o)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (blockIdx.x == gridDim.x - 1)
      for (int c = 0; c < 4; ++c) last[c] = sh[c][0];
    if (!isfinite(sh[0][0]) || !isfinite(sh[1][0]) || !isfinite(sh[2][0]) || !isfinite(sh[3][0]))
      last[4] = 1.0;
    if (t < cap)
      for (int c = 0; c < 3; ++c) hist[t * 3 + c] = sh[c][0];
  }
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

struct Layout3 {
  int pitch, ntx, nblocks;
  int64_t plane;
  size_t A, B, links, rowf, part, last, hist, total;
};

size_t esz(int precision) { return precision == LBM_FP64 ? 8 : 4; }

Layout3 layout3(const lbm3d_params& p) {
  Layout3 L;
  L.pitch = (p.nx + 63) / 64 * 64;
  L.ntx = (p.nx + kB3 - 1) / kB3;
  L.nblocks = L.ntx * ((p.ny * p.nz + kR3 - 1) / kR3);
  L.plane = int64_t(p.nz) * p.ny * L.pitch;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += al256(b);
    return at;
  };
  L.A = take(size_t(19) * L.plane * esz(p.precision));
  L.B = take(size_t(19) * L.plane * esz(p.precision));
  L.links = take(size_t(L.plane) * 4);
  L.rowf = take(size_t(p.nz) * p.ny);
  L.part = take(size_t(kRing) * L.nblocks * 4 * 8);
  L.last = take(8 * 8);
  L.hist = take(size_t(p.history_cap) * 3 * 8);
  L.total = o;
  return L;
}

lbm_status check3(const lbm3d_params* p) {
  if (!p) return set_error(LBM_EINVAL, "params is NULL");
  if (p->nx < 4 || p->ny < 4 || p->nz < 4) return set_error(LBM_EINVAL, "nx, ny, nz must be >= 4");
  if (int64_t(p->nx) * p->ny * p->nz >= (int64_t(1) << 31) / 2)
    return set_error(LBM_EINVAL, "lattice too large");
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32_OFFSET)
    return set_error(LBM_EINVAL, "precision must be LBM_FP64 or LBM_FP32_OFFSET");
  for (int32_t b : {p->lateral_y, p->lateral_z})
    if (b != LBM_LATERAL_WALLS && b != LBM_LATERAL_PERIODIC) return set_error(LBM_EINVAL, "bad lateral");
  if (p->xbc != LBM_X_INOUT && p->xbc != LBM_X_PERIODIC) return set_error(LBM_EINVAL, "bad xbc");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return set_error(LBM_EINVAL, "tau must be > 1/2");
  if (!(std::fabs(p->u_in) < 0.5)) return set_error(LBM_EINVAL, "|u_in| must be < 0.5");
  if (!(p->rho_out > 0.0) || !std::isfinite(p->rho_out)) return set_error(LBM_EINVAL, "rho_out must be > 0");
  if (p->history_cap < 0) return set_error(LBM_EINVAL, "history_cap < 0");
  return LBM_OK;
}

#define L3_TRY(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return set_error(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm3d_ctx {
  lbm3d_params p;
  hipStream_t stream;
  Layout3 L;
  char* base;
  bool has_geometry = false;
  int cur = 0;              // which buffer holds the state: 0 = A, 1 = B
  int64_t t = 0;
  int64_t pending = 0;      // steps whose partials are not yet reduced

  // reduce the partials of the pending steps (one workgroup per step)
  lbm_status flush() {
    if (pending) {
      hipLaunchKernelGGL(k3_reduce, dim3(unsigned(pending)), dim3(kRed3), 0, stream,
                         reinterpret_cast<const double*>(base + L.part), L.nblocks,
                         reinterpret_cast<double*>(base + L.last),
                         reinterpret_cast<double*>(base + L.hist), t - pending,
                         int64_t(p.history_cap));
      pending = 0;
      L3_TRY(hipGetLastError());
    }
    return LBM_OK;
  }
  std::vector<uint8_t> mask;

  size_t bufoff(int which) const { return which == 0 ? L.A : L.B; }

  // host populations (absolute, [q][z][y][x]) -> both device buffers
  lbm_status upload(const std::vector<double>& f) {
    const size_t e = esz(p.precision);
    const size_t n = size_t(19) * L.plane;
    std::vector<char> h(n * e, 0);
    const size_t nx = p.nx, ny = p.ny, nz = p.nz;
    for (size_t q = 0; q < 19; ++q) {
      const double w = w3<double>(int(q));
      for (size_t z = 0; z < nz; ++z)
        for (size_t y = 0; y < ny; ++y)
          for (size_t x = 0; x < nx; ++x) {
            const double g = f[((q * nz + z) * ny + y) * nx + x] - w;
            const size_t d = q * L.plane + (z * ny + y) * L.pitch + x;
            if (e == 8) reinterpret_cast<double*>(h.data())[d] = g;
            else reinterpret_cast<float*>(h.data())[d] = float(g);
          }
    }
    L3_TRY(hipMemcpyAsync(base + L.A, h.data(), h.size(), hipMemcpyHostToDevice, stream));
    L3_TRY(hipMemcpyAsync(base + L.B, h.data(), h.size(), hipMemcpyHostToDevice, stream));
    L3_TRY(hipStreamSynchronize(stream));
    cur = 0;
    return LBM_OK;
  }

  std::vector<double> equilibrium_state(const double* rho, const double* u) const {
    const size_t nx = p.nx, ny = p.ny, nz = p.nz, nn = nx * ny * nz;
    std::vector<double> f(19 * nn);
    for (size_t i = 0; i < nn; ++i) {
      const bool solid = mask[i] != 0;
      const double r = solid ? 1.0 : (rho ? rho[i] : 1.0);
      const double ux = solid ? 0.0 : (u ? u[i] : p.u_in);
      const double uy = solid || !u ? 0.0 : u[nn + i];
      const double uz = solid || !u ? 0.0 : u[2 * nn + i];
      const double usq = ux * ux + uy * uy + uz * uz;
      for (int q = 0; q < 19; ++q) {
        const double cu = c3(q, 0) * ux + c3(q, 1) * uy + c3(q, 2) * uz;
        f[q * nn + i] = w3<double>(q) * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      }
    }
    return f;
  }
};

extern "C" {

size_t lbm3d_workspace_bytes(const lbm3d_params* p) {
  if (check3(p)) return 0;
  return layout3(*p).total;
}

lbm_status lbm3d_create(const lbm3d_params* p, void* ws, size_t bytes, lbm3d_ctx** out) {
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status s = check3(p);
  if (s) return s;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256)
    return set_error(LBM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  const Layout3 L = layout3(*p);
  if (bytes < L.total) return set_error(LBM_ENOSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);
  lbm3d_ctx* c = new lbm3d_ctx();
  c->p = *p;
  c->stream = static_cast<hipStream_t>(p->stream);
  c->L = L;
  c->base = static_cast<char*>(ws);
  *out = c;
  return LBM_OK;
}

lbm_status lbm3d_destroy(lbm3d_ctx* c) {
  if (c) (void)hipStreamSynchronize(c->stream);
  delete c;
  return LBM_OK;
}

lbm_status lbm3d_set_geometry(lbm3d_ctx* c, const uint8_t* host_mask) {
  if (!c || !host_mask) return set_error(LBM_EINVAL, "NULL argument");
  const lbm3d_params& p = c->p;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const size_t nn = size_t(nx) * ny * nz;
  for (size_t i = 0; i < nn; ++i)
    if (host_mask[i] > 1) return set_error(LBM_EINVAL, "mask values must be 0 (fluid) or 1 (body)");
  if (p.xbc == LBM_X_INOUT)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        if (host_mask[(size_t(z) * ny + y) * nx] || host_mask[(size_t(z) * ny + y) * nx + nx - 1])
          return set_error(LBM_EINVAL, "the planes x = 0 and x = nx-1 must be fluid");
  c->mask.assign(host_mask, host_mask + nn);
  const bool xper = p.xbc == LBM_X_PERIODIC, yper = p.lateral_y == LBM_LATERAL_PERIODIC,
             zper = p.lateral_z == LBM_LATERAL_PERIODIC;
  std::vector<uint32_t> links(size_t(c->L.plane), 0);
  std::vector<uint8_t> rowf(size_t(nz) * ny, 0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t i = (size_t(z) * ny + y) * nx + x;
        uint32_t lk = host_mask[i] ? kSolid3 : 0u;
        for (int q = 1; q < 19; ++q) {
          int sx = x - c3(q, 0), sy = y - c3(q, 1), sz = z - c3(q, 2);
          if (sx < 0 || sx >= nx) {
            if (!xper) continue;
            sx = (sx + nx) % nx;
          }
          if (sy < 0 || sy >= ny) {
            if (!yper) continue;
            sy = (sy + ny) % ny;
          }
          if (sz < 0 || sz >= nz) {
            if (!zper) continue;
            sz = (sz + nz) % nz;
          }
          if (host_mask[(size_t(sz) * ny + sy) * nx + sx]) lk |= 1u << q;
        }
        links[(size_t(z) * ny + y) * c->L.pitch + x] = lk;
        if (lk) rowf[size_t(z) * ny + y] = 1;
      }
  L3_TRY(hipMemcpyAsync(c->base + c->L.links, links.data(), links.size() * 4, hipMemcpyHostToDevice,
                        c->stream));
  L3_TRY(hipMemcpyAsync(c->base + c->L.rowf, rowf.data(), rowf.size(), hipMemcpyHostToDevice,
                        c->stream));
  L3_TRY(hipMemsetAsync(c->base + c->L.last, 0, 8 * 8, c->stream));
  c->has_geometry = true;
  c->t = 0;
  c->pending = 0;
  return c->upload(c->equilibrium_state(nullptr, nullptr));
}

lbm_status lbm3d_init_fields(lbm3d_ctx* c, const double* rho, const double* u) {
  if (!c || !rho || !u) return set_error(LBM_EINVAL, "NULL argument");
  if (!c->has_geometry) return set_error(LBM_ESTATE, "set the geometry first");
  return c->upload(c->equilibrium_state(rho, u));
}

lbm_status lbm3d_step(lbm3d_ctx* c, int64_t nsteps) {
  if (!c) return set_error(LBM_EINVAL, "NULL context");
  if (!c->has_geometry) return set_error(LBM_ESTATE, "set the geometry first");
  if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps < 0");
  const lbm3d_params& p = c->p;
  const Layout3& L = c->L;
  Step3 s;
  s.links = reinterpret_cast<const uint32_t*>(c->base + L.links);
  s.rowf = reinterpret_cast<const uint8_t*>(c->base + L.rowf);
  s.part = reinterpret_cast<double*>(c->base + L.part);
  s.nx = p.nx;
  s.ny = p.ny;
  s.nz = p.nz;
  s.pitch = L.pitch;
  s.ntx = L.ntx;
  s.nblocks = L.nblocks;
  {
    const int64_t row = int64_t(L.pitch) * int64_t(esz(p.precision));
    s.chunk = int(std::max<int64_t>(1, ((int64_t(512) << 10) + row / 2) / row)) * L.ntx;
  }
  s.plane = L.plane;
  s.xper = p.xbc == LBM_X_PERIODIC;
  s.yper = p.lateral_y == LBM_LATERAL_PERIODIC;
  s.zper = p.lateral_z == LBM_LATERAL_PERIODIC;
  s.omega = 1.0 / p.tau;
  s.u_in = p.u_in;
  s.one_minus_rho_out = 1.0 - p.rho_out;
  double* ring = reinterpret_cast<double*>(c->base + L.part);
  for (int64_t i = 0; i < nsteps; ++i) {
    s.A = c->base + c->bufoff(c->cur);
    s.B = c->base + c->bufoff(1 - c->cur);
    s.part = ring + (c->t % kRing) * int64_t(L.nblocks) * 4;
    if (p.precision == LBM_FP64)
      hipLaunchKernelGGL(k3_step<double>, dim3(L.nblocks), dim3(kT3), 0, c->stream, s);
    else
      hipLaunchKernelGGL(k3_step<float>, dim3(L.nblocks), dim3(kT3), 0, c->stream, s);
    c->cur = 1 - c->cur;
    ++c->t;
    if (++c->pending == kRing) {
      lbm_status st = c->flush();
      if (st) return st;
    }
  }
  L3_TRY(hipGetLastError());
  return LBM_OK;
}

lbm_status lbm3d_forces(lbm3d_ctx* c, lbm3d_force_out* out) {
  if (!c || !out) return set_error(LBM_EINVAL, "NULL argument");
  double h[8];
  lbm_status st = c->flush();
  if (st) return st;
  L3_TRY(hipStreamSynchronize(c->stream));
  L3_TRY(hipMemcpy(h, c->base + c->L.last, sizeof(h), hipMemcpyDeviceToHost));
  out->fx = h[0];
  out->fy = h[1];
  out->fz = h[2];
  out->dmass = h[3];
  out->step = c->t;
  out->nonfinite = h[4] != 0.0;
  out->reserved = 0;
  return out->nonfinite ? set_error(LBM_EUNSTABLE, "a non-finite value appeared") : LBM_OK;
}

lbm_status lbm3d_force_history(lbm3d_ctx* c, double* fx, double* fy, double* fz, int64_t cap,
                               int64_t* n) {
  if (!c || !fx || !fy || !fz || !n || cap < 0) return set_error(LBM_EINVAL, "bad argument");
  const int64_t m = std::min(std::min(cap, c->t), int64_t(c->p.history_cap));
  std::vector<double> h(size_t(m) * 3);
  lbm_status st = c->flush();
  if (st) return st;
  L3_TRY(hipStreamSynchronize(c->stream));
  if (m) L3_TRY(hipMemcpy(h.data(), c->base + c->L.hist, h.size() * 8, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < m; ++i) {
    fx[i] = h[3 * i];
    fy[i] = h[3 * i + 1];
    fz[i] = h[3 * i + 2];
  }
  *n = m;
  return LBM_OK;
}

lbm_status lbm3d_read_populations(lbm3d_ctx* c, double* host) {
  if (!c || !host) return set_error(LBM_EINVAL, "NULL argument");
  if (!c->has_geometry) return set_error(LBM_ESTATE, "set the geometry first");
  const lbm3d_params& p = c->p;
  const size_t e = esz(p.precision), n = size_t(19) * c->L.plane;
  std::vector<char> h(n * e);
  L3_TRY(hipStreamSynchronize(c->stream));
  L3_TRY(hipMemcpy(h.data(), c->base + c->bufoff(c->cur), h.size(), hipMemcpyDeviceToHost));
  const size_t nx = p.nx, ny = p.ny, nz = p.nz;
  for (size_t q = 0; q < 19; ++q) {
    const double w = w3<double>(int(q));
    for (size_t z = 0; z < nz; ++z)
      for (size_t y = 0; y < ny; ++y)
        for (size_t x = 0; x < nx; ++x) {
          const size_t d = q * c->L.plane + (z * ny + y) * c->L.pitch + x;
          const double g = e == 8 ? reinterpret_cast<double*>(h.data())[d]
                                  : double(reinterpret_cast<float*>(h.data())[d]);
          host[((q * nz + z) * ny + y) * nx + x] = g + w;
        }
  }
  return LBM_OK;
}

lbm_status lbm3d_write_populations(lbm3d_ctx* c, const double* host) {
  if (!c || !host) return set_error(LBM_EINVAL, "NULL argument");
  if (!c->has_geometry) return set_error(LBM_ESTATE, "set the geometry first");
  const size_t n = size_t(19) * c->p.nx * c->p.ny * c->p.nz;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) return set_error(LBM_EINVAL, "non-finite population");
  return c->upload(std::vector<double>(host, host + n));
}

lbm_status lbm3d_sync(lbm3d_ctx* c) {
  if (!c) return set_error(LBM_EINVAL, "NULL context");
  lbm_status st = c->flush();
  if (st) return st;
  L3_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

}  // extern "C"
