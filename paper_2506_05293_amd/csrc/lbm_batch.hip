// Batched launch over many uneven D2Q9 lattices (C ABI of
// include/lbm_batch.h).
//
// Work is split into row items: 64 columns of one row of one lattice, one
// node per lane (LBM_BATCH_SCALAR, the default), or 256 columns with four
// nodes per lane and 16-byte accesses (LBM_BATCH_SCALAR=0).  Every item is
// updated with the node code of the single-lattice kernel (FP32 offsets),
// logging the pre-collision populations of the logged columns on logging
// steps.  The item list is dealt to the XCDs in chunks of kItemChunk
// consecutive items (XCD x takes chunks x, x + 8, ...), so the items that
// share edge cache lines meet in one L2 and the eight XCDs work on nearby
// addresses at any time (one contiguous eighth of the list per XCD measured
// 6.7 % slower on the 64-pair batch: the XCDs' concurrent rows then sit at
// arbitrary spacings, which load the HBM channels unevenly).
//
// One launch per step (k_batch_step, the default mode): every wave takes one
// item; the workgroups first reduce the partial sums of the previous step
// for lattices w, w + G, ... (FP64, fixed item order) into that lattice's
// accumulators and force history and retire a lattice whose force or mass
// is no longer finite; k_batch_flush reduces the last step of a call.
//
// Persistent mode (k_batch): one cooperative grid of resident workgroups
// advances every lattice for a number of steps; per step the same reduction,
// then every wave strides on its own over its XCD's items, then a grid
// barrier, whose wait is bounded: a workgroup that waits longer than the
// spin limit raises the error flag and leaves, and every workgroup leaves
// once the flag is up, so the grid always drains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/lbm_batch.h"
#include "d2q9_dev.hpp"
#include "lbm_internal.hpp"
#include "node_dev.hpp"

namespace lbm {
namespace {

constexpr int kDefaultSpin = 1 << 22;   // polls of ~50 ns: ~0.2 s per barrier
constexpr int kBatchGroupsPerCu = 4;
// s_waitcnt operand (gfx9 encoding) that waits for vmcnt = 0 only:
// vmcnt bits [3:0] and [15:14] zero, expcnt [6:4] and lgkmcnt [11:8] at their maximum
constexpr int kWaitVmcnt0 = 0x0F70;
#ifndef LBM_BATCH_SCALAR
#define LBM_BATCH_SCALAR 1
#endif
constexpr int kItemChunk = 128;         // items per chunk dealt to an XCD (64 to 512 measured alike)

// The k-th item of XCD x (increasing in k).
__device__ __forceinline__ int xcd_item(int x, int k) {
  return ((k / kItemChunk) * 8 + x) * kItemChunk + k % kItemChunk;
}

// Fields of one lattice read by bulk_node, with A/B chosen per step.
struct LatView {
  const float* A;
  float* B;
  const uint32_t* links;
  const uint8_t* chunk;
  const double* inlet;
  int nx, ny, pitch, nchunk;
  int64_t plane;
  int xper, yper, n_nn;
  double omega, s_e, s_eps, s_q, u_in, one_minus_rho_out;
};

struct BatchLat {
  float* buf[2];
  const uint32_t* links;
  const uint8_t* chunk;
  int nx, ny, pitch, nchunk;
  int64_t plane;
  double omega, s_q, u_in, one_minus_rho_out, n_fluid;
  int item0, nitems;           // this lattice's range of the item table
  int log_role, log_x, log_row0, pad;
};

struct BatchCtl {              // device-side control words
  unsigned count, gen;
  int err;
  unsigned seen;               // arrivals counted when a wait gave up
};

struct BatchArgs {
  const BatchLat* lats;
  const int4* items;           // (lattice, chunk column, row, sub): 64 x 1 nodes
                               // (256 x 1 with the four-nodes-per-lane code)
  int nlat, nitems;
  int xper, yper;
  double s_e, s_eps;
  float* part[2];              // [nitems][4] per step parity (fx, fy, drho, 0)
  Acc* acc;                    // [nlat]
  double* hist;                // [nlat][hist_cap][3]
  int64_t hist_cap;
  int* retired;                // [nlat]
  BatchCtl* ctl;
  int spin_limit;
  int64_t step0, nsteps;       // steps taken before this launch, steps to take
  int64_t log_start, log_every, log_slots;
  int log_rows;
  float* x;                    // data set: [slots * log_rows][27]
  float* xa;                   // ablation inputs [slots * log_rows][27]
  float* t;                    // targets [slots * log_rows][3] (raw f(log_x) until fixed)
};

// Logging observer of the pre-collision populations (offsets).
struct LogHook {
  float* x;
  float* xa;
  float* t;
  int role, log_x;
  int64_t row_base;            // sample index of row 0, or -1: not a logging step
  __device__ void operator()(int x, int y, const float* g) const {
    if (row_base < 0 || role == 0) return;
    const int64_t s = row_base + y;
    const int j = log_x - 1 - x;
    if (j >= 0 && j < 3) {
      float* d = (role == 1 ? this->x : xa) + s * 27 + 9 * j;
#pragma unroll
      for (int q = 0; q < 9; ++q) d[q] = g[q];
    } else if (role == 1 && x == log_x) {
      t[s * 3 + 0] = g[3];
      t[s * 3 + 1] = g[6];
      t[s * 3 + 2] = g[7];
    }
  }
};

__device__ void block_sum4_d(double s[4], double out[4]) {
  __shared__ double red[kWaves][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = wave_sum(s[k]);
  __syncthreads();
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

// Fixed-order FP64 sum of lattice l's item partials of one step, committed to
// its accumulators (and its retirement flag).
__device__ void reduce_lattice(const BatchArgs& a, int l, const float* part) {
  const BatchLat& d = a.lats[l];
  double s[4] = {0.0, 0.0, 0.0, 0.0}, t[4];
  for (int k = threadIdx.x; k < d.nitems; k += kBlock) {
    const float4 p = reinterpret_cast<const float4*>(part)[d.item0 + k];
    s[0] += double(p.x);
    s[1] += double(p.y);
    s[2] += double(p.z);
  }
  block_sum4_d(s, t);
  if (threadIdx.x == 0) {
    Acc* acc = a.acc + l;
    acc->fx = t[0];
    acc->fy = t[1];
    acc->fx_sum += t[0];
    acc->fy_sum += t[1];
    acc->mass = d.n_fluid + t[2];
    const bool bad = !isfinite(t[0]) || !isfinite(t[1]) || !isfinite(t[2]);
    if (bad) {
      acc->nonfinite = 1;
      a.retired[l] = 1;
    }
    const int64_t n = acc->n_reduced;
    if (n < a.hist_cap) {
      double* h = a.hist + (int64_t(l) * a.hist_cap + n) * 3;
      h[0] = t[0];
      h[1] = t[1];
      h[2] = d.n_fluid + t[2];
    }
    acc->n_reduced = n + 1;
  }
}

// Grid-wide barrier with a bounded wait.  Returns false (on every thread of
// the workgroup) if the wait timed out or another workgroup raised the flag.
// The L2 caches of the eight XCDs are not coherent with each other, and the
// next step reads populations written on other XCDs.  Every wave first waits
// until its own stores are complete in its XCD's L2 (s_waitcnt vmcnt(0));
// after the workgroup barrier one thread makes them visible device-wide (a
// device-scope release: write-back of the L2's dirty lines) before it
// arrives, and after the last arrival takes a device-scope acquire
// (invalidation of this CU's L1 and of the XCD's L2), which covers every wave
// of the workgroup: they share the CU, and none of them loads in between.
// A release per wave would repeat the L2 write-back once per wave.
__device__ bool grid_barrier(const BatchArgs& a) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    BatchCtl* c = a.ctl;
    int good = 1;
    const unsigned g = __hip_atomic_load(&c->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = atomicAdd(&c->count, 1u);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(&c->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&c->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int spins = 0;
      // relaxed polls: an acquire per poll would invalidate the L2 under the
      // waves still streaming; the acquire fence below follows the wait
      while (__hip_atomic_load(&c->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++spins > a.spin_limit ||
            __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          if (!__hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&c->seen, __hip_atomic_load(&c->count, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT));
          atomicExch(&c->err, 1);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (__hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) good = 0;
    ok = good;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

// Read-only tables of the launch, read through the constant address space so
// that wave-uniform loads from them are scalar loads.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T*;

// Optional occupancy request (waves per SIMD) for the batched kernel.
#ifdef LBM_BATCH_WAVES_PER_EU
#define LBM_BATCH_ATTR \
  __attribute__((amdgpu_waves_per_eu(LBM_BATCH_WAVES_PER_EU, LBM_BATCH_WAVES_PER_EU)))
#else
#define LBM_BATCH_ATTR
#endif

// One row item (64 or 256 columns of one lattice row) of step gs by one wave:
// the node update, then the wave's partial (fx, fy, sum rho - 1).
template <int MRT>
__device__ __forceinline__ void batch_item(const BatchArgs& a, int it, int par, int64_t slot,
                                           int lane) {
  const const_ptr<int> items = (const_ptr<int>)(a.items);
  const const_ptr<BatchLat> lats = (const_ptr<BatchLat>)(a.lats);
  const int lat = items[4 * it], tx = items[4 * it + 1], y = items[4 * it + 2];
  const const_ptr<BatchLat> d = lats + lat;
  float fx = 0.f, fy = 0.f, dm = 0.f;
  if (!a.retired[lat]) {
    LatView v;
    v.A = d->buf[par];
    v.B = d->buf[par ^ 1];
    v.links = d->links;
    v.chunk = d->chunk;
    v.inlet = nullptr;
    v.nx = d->nx;
    v.ny = d->ny;
    v.pitch = d->pitch;
    v.nchunk = d->nchunk;
    v.plane = d->plane;
    v.xper = a.xper;
    v.yper = a.yper;
    v.n_nn = 0;
    v.omega = d->omega;
    v.s_e = a.s_e;
    v.s_eps = a.s_eps;
    v.s_q = d->s_q;
    v.u_in = d->u_in;
    v.one_minus_rho_out = d->one_minus_rho_out;
    LogHook hook{a.x, a.xa, a.t, d->log_role, d->log_x,
                 slot < 0 ? int64_t(-1) : slot * a.log_rows + d->log_row0};
#if LBM_BATCH_SCALAR
    const int x = tx * kChunk + items[4 * it + 3] * 64 + lane;
    if (x < v.nx) bulk_node<float, MRT>(v, tx, x, y, fx, fy, dm, hook);
#else
    bulk_row<float, MRT>(v, tx, y, lane, fx, fy, dm, hook);
#endif
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  dm = wave_sum(dm);
  if (lane == 0) reinterpret_cast<float4*>(a.part[par])[it] = make_float4(fx, fy, dm, 0.f);
}

// The logging slot of the step taken after gs steps, or -1.
__device__ __forceinline__ int64_t log_slot(const BatchArgs& a, int64_t gs) {
  if (gs < a.log_start || (gs - a.log_start) % a.log_every != 0) return -1;
  const int64_t slot = (gs - a.log_start) / a.log_every;
  return slot < a.log_slots ? slot : -1;
}

template <int MRT>
__global__ void __launch_bounds__(kBlock) LBM_BATCH_ATTR k_batch(const BatchArgs a) {
  // this wave's share of the items: XCD x = blockIdx % 8 takes its chunks
  // of the list (xcd_item); its waves stride over them
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int lane = int(threadIdx.x & 63);
  const int xcd = int(blockIdx.x & 7);
  const int groups = int(gridDim.x) >> 3;            // workgroups per XCD (grid % 8 == 0)
  const int stride = groups * kWaves;
  const int start = int(blockIdx.x >> 3) * kWaves + wave;
  for (int64_t s = 0; s < a.nsteps; ++s) {
    const int64_t gs = a.step0 + s;         // steps taken before this one
    const int par = int(gs & 1);
    // 1. the previous step's sums (pipelined into this step)
    if (s > 0)
      for (int l = blockIdx.x; l < a.nlat; l += gridDim.x) reduce_lattice(a, l, a.part[par ^ 1]);
    // 2. all row items
    const int64_t slot = log_slot(a, gs);
    for (int k = start; xcd_item(xcd, k) < a.nitems; k += stride)
      batch_item<MRT>(a, xcd_item(xcd, k), par, slot, lane);
    // 3. all nodes of this step written before any of the next is read
    if (!grid_barrier(a)) return;
  }
  // flush: the last step's sums
  const int last = int((a.step0 + a.nsteps - 1) & 1);
  for (int l = blockIdx.x; l < a.nlat; l += gridDim.x) reduce_lattice(a, l, a.part[last]);
}

// One step per launch (the kernel boundary orders the steps): wave w of
// workgroup b takes item (b / 8) * 4 + w of XCD b % 8 (xcd_item);
// the workgroups first reduce the previous step's partials when that step
// was taken by the previous launch of the same call.
template <int MRT>
__global__ void __launch_bounds__(kBlock) k_batch_step(const BatchArgs a, int reduce_prev) {
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int lane = int(threadIdx.x & 63);
  const int xcd = int(blockIdx.x & 7);
  const int64_t gs = a.step0;
  const int par = int(gs & 1);
  if (reduce_prev)
    for (int l = blockIdx.x; l < a.nlat; l += gridDim.x) reduce_lattice(a, l, a.part[par ^ 1]);
  const int it = xcd_item(xcd, int(blockIdx.x >> 3) * kWaves + wave);
  if (it < a.nitems) batch_item<MRT>(a, it, par, log_slot(a, gs), lane);
}

// The sums of the last step of a call (parity par).
__global__ void __launch_bounds__(kBlock) k_batch_flush(const BatchArgs a, int par) {
  for (int l = blockIdx.x; l < a.nlat; l += gridDim.x) reduce_lattice(a, l, a.part[par]);
}

// t -= x[column log_x - 1] for the samples of slots [s0, s1).
__global__ void k_fix_targets(float* t, const float* x, int64_t n0, int64_t n1) {
  const int64_t i = n0 + int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n1) return;
  t[i * 3 + 0] -= x[i * 27 + 3];
  t[i * 3 + 1] -= x[i * 27 + 6];
  t[i * 3 + 2] -= x[i * 27 + 7];
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_batch {
  lbm_batch_params p;
  hipStream_t stream;
  int nlat, nitems;
  std::vector<BatchLat> lat;        // host copy of the descriptors
  BatchArgs args;
  int grid;                         // persistent grid
  int grid_step;                    // per-step grid: one wave per item
  int64_t steps;
  int64_t fixed_slots;              // slots whose targets are already corrections
};

namespace {

struct BatchLayout {
  std::vector<size_t> buf0, buf1, links, chunk;
  size_t lats, items, part0, part1, acc, hist, retired, ctl, x, xa, t, total;
  int nitems;
};

BatchLayout batch_layout(const lbm_batch_params& p, const lbm_batch_lattice* lat, int n) {
  BatchLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = o;
    o = align256(o + b);
    return at;
  };
  L.nitems = 0;
  for (int i = 0; i < n; ++i) {
    const int pitch = int(align256(size_t(lat[i].nx)));
    const int nch = pitch / kChunk;
    const size_t plane = size_t(lat[i].ny) * pitch;
    L.buf0.push_back(take(9 * plane * 4));
    L.buf1.push_back(take(9 * plane * 4));
    L.links.push_back(take(plane * 4));
    L.chunk.push_back(take(size_t(lat[i].ny) * nch));
#if LBM_BATCH_SCALAR
    L.nitems += (lat[i].nx + 63) / 64 * lat[i].ny;
#else
    L.nitems += nch * lat[i].ny;
#endif
  }
  L.lats = take(sizeof(BatchLat) * size_t(n));
  L.items = take(sizeof(int4) * size_t(L.nitems));
  L.part0 = take(size_t(L.nitems) * 16);
  L.part1 = take(size_t(L.nitems) * 16);
  L.acc = take(sizeof(Acc) * size_t(n));
  L.hist = take(size_t(std::max<int64_t>(p.history_cap, 0)) * 24 * size_t(n));
  L.retired = take(4 * size_t(n));
  L.ctl = take(sizeof(BatchCtl));
  const size_t samples = size_t(std::max<int64_t>(p.log_slots, 0)) * size_t(std::max(p.log_rows, 0));
  L.x = take(samples * 27 * 4);
  L.xa = take(samples * 27 * 4);
  L.t = take(samples * 3 * 4);
  L.total = o;
  return L;
}

lbm_status check_batch(const lbm_batch_params* p, const lbm_batch_lattice* lat, int n) {
  if (!p || !lat) return set_error(LBM_EINVAL, "NULL argument");
  if (n < 1) return set_error(LBM_EINVAL, "need at least one lattice");
  if (p->collision != LBM_BGK && p->collision != LBM_MRT) return set_error(LBM_EINVAL, "bad collision");
  if (p->lateral != LBM_LATERAL_WALLS && p->lateral != LBM_LATERAL_PERIODIC)
    return set_error(LBM_EINVAL, "bad lateral");
  if (p->history_cap < 0 || p->log_slots < 0 || p->log_rows < 0 || p->log_start < 0)
    return set_error(LBM_EINVAL, "negative size");
  if (p->log_slots > 0 && p->log_every < 1) return set_error(LBM_EINVAL, "log_every must be >= 1");
  if (p->spin_limit < 0) return set_error(LBM_EINVAL, "spin_limit < 0");
  if (p->groups_per_cu < 0) return set_error(LBM_EINVAL, "groups_per_cu < 0");
  if (p->launch != LBM_BATCH_PERSISTENT && p->launch != LBM_BATCH_PER_STEP)
    return set_error(LBM_EINVAL, "bad launch mode");
  for (int i = 0; i < n; ++i) {
    const lbm_batch_lattice& L = lat[i];
    if (L.nx < 8 || L.ny < 8) return set_error(LBM_EINVAL, "lattice %d: nx, ny must be >= 8", i);
    if ((int64_t(L.nx) + 255) * L.ny * 8 >= (int64_t(1) << 32))
      return set_error(LBM_EINVAL, "lattice %d too large", i);
    if (!(L.tau > 0.5)) return set_error(LBM_EINVAL, "lattice %d: tau must be > 0.5", i);
    if (!(std::fabs(L.u_in) < 0.5) || !(L.rho_out > 0))
      return set_error(LBM_EINVAL, "lattice %d: bad u_in or rho_out", i);
    if (!L.mask) return set_error(LBM_EINVAL, "lattice %d: mask is NULL", i);
    if (L.log_role < 0 || L.log_role > 2) return set_error(LBM_EINVAL, "lattice %d: bad log_role", i);
    if (L.log_role) {
      const int lo = L.log_role == 1 ? 4 : 3;
      if (L.log_x < lo || L.log_x > L.nx - 1) return set_error(LBM_EINVAL, "lattice %d: bad log_x", i);
      if (L.log_row0 < 0 || int64_t(L.log_row0) + L.ny > p->log_rows)
        return set_error(LBM_EINVAL, "lattice %d: rows exceed log_rows", i);
    }
  }
  return LBM_OK;
}

#define BTRY(expr)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return set_error(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

lbm_status batch_sync(lbm_batch* b) {
  BTRY(hipStreamSynchronize(b->stream));
  BatchCtl ctl;
  BTRY(hipMemcpy(&ctl, b->args.ctl, sizeof ctl, hipMemcpyDeviceToHost));
  if (ctl.err)
    return set_error(LBM_EHIP,
                     "batch barrier wait exceeded its bound (%u of %d workgroups had arrived); "
                     "the batch state is void", ctl.seen, b->grid);
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_batch_params* p, const lbm_batch_lattice* lat, int32_t n) {
  if (check_batch(p, lat, n) != LBM_OK) return 0;
  return batch_layout(*p, lat, n).total;
}

lbm_status lbm_batch_create(const lbm_batch_params* p, const lbm_batch_lattice* lat, int32_t n,
                            void* ws, size_t bytes, lbm_batch** out) {
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status st = check_batch(p, lat, n);
  if (st) return st;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256)
    return set_error(LBM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  const BatchLayout L = batch_layout(*p, lat, n);
  if (bytes < L.total) return set_error(LBM_ENOSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);
  for (int i = 0; i < n; ++i) {
    for (int y = 0; y < lat[i].ny; ++y)
      if (lat[i].mask[int64_t(y) * lat[i].nx] || lat[i].mask[int64_t(y) * lat[i].nx + lat[i].nx - 1])
        return set_error(LBM_EINVAL, "lattice %d: columns 0 and nx-1 must be fluid", i);
    for (int64_t k = 0; k < int64_t(lat[i].nx) * lat[i].ny; ++k)
      if (lat[i].mask[k] > 2) return set_error(LBM_EINVAL, "lattice %d: mask value > 2", i);
  }
  char* base = static_cast<char*>(ws);
  hipStream_t stream = static_cast<hipStream_t>(p->stream);
  const bool yper = p->lateral == LBM_LATERAL_PERIODIC;

  lbm_batch* b = new lbm_batch();
  b->p = *p;
  b->stream = stream;
  b->nlat = n;
  b->nitems = L.nitems;
  std::vector<int4> items;
  items.reserve(L.nitems);
  auto cleanup = [&](lbm_status s) {
    delete b;
    return s;
  };
  for (int i = 0; i < n; ++i) {
    const lbm_batch_lattice& q = lat[i];
    BatchLat d{};
    d.pitch = int(align256(size_t(q.nx)));
    d.nchunk = d.pitch / kChunk;
    d.nx = q.nx;
    d.ny = q.ny;
    d.plane = int64_t(q.ny) * d.pitch;
    d.buf[0] = reinterpret_cast<float*>(base + L.buf0[i]);
    d.buf[1] = reinterpret_cast<float*>(base + L.buf1[i]);
    d.links = reinterpret_cast<const uint32_t*>(base + L.links[i]);
    d.chunk = reinterpret_cast<const uint8_t*>(base + L.chunk[i]);
    d.omega = 1.0 / q.tau;
    d.s_q = p->s_q > 0 ? p->s_q : 1.0 / (0.5 + (3.0 / 16.0) / (q.tau - 0.5));
    d.u_in = q.u_in;
    d.one_minus_rho_out = 1.0 - q.rho_out;
    d.item0 = int(items.size());
    for (int y = 0; y < q.ny; ++y)
      for (int tx = 0; tx < d.nchunk; ++tx)
#if LBM_BATCH_SCALAR
        for (int sub = 0; sub < kChunk / 64; ++sub)
          if (tx * kChunk + sub * 64 < q.nx) items.push_back(make_int4(i, tx, y, sub));
#else
        items.push_back(make_int4(i, tx, y, 0));
#endif
    d.nitems = int(items.size()) - d.item0;
    d.log_role = q.log_role;
    d.log_x = q.log_x;
    d.log_row0 = q.log_row0;
    std::vector<uint32_t> links(size_t(d.plane), 0u);
    std::vector<uint8_t> chunk(size_t(q.ny) * d.nchunk, 0);
    d.n_fluid = double(build_links(q.mask, q.nx, q.ny, d.pitch, d.nchunk, false, yper, links.data(),
                                   chunk.data()));
    hipError_t e = hipMemcpyAsync(const_cast<uint32_t*>(d.links), links.data(), links.size() * 4,
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(const_cast<uint8_t*>(d.chunk), chunk.data(), chunk.size(),
                         hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);   // host vectors go out of scope
    if (e != hipSuccess) return cleanup(set_error(LBM_EHIP, "geometry upload: %s", hipGetErrorString(e)));
    InitLaunch I{};
    I.precision = LBM_FP32_OFFSET;
    I.A = d.buf[0];
    I.B = d.buf[1];
    I.links = d.links;
    I.nx = q.nx;
    I.ny = q.ny;
    I.pitch = d.pitch;
    I.plane = d.plane;
    I.y0 = 0;
    I.rows = q.ny;
    I.fields = nullptr;
    I.u_in = q.u_in;
    I.noise_amp = p->noise_amp;
    I.seed = q.seed;
    e = launch_init(I, stream);
    if (e != hipSuccess) return cleanup(set_error(LBM_EHIP, "init: %s", hipGetErrorString(e)));
    b->lat.push_back(d);
  }
  hipError_t e = hipMemcpyAsync(base + L.lats, b->lat.data(), sizeof(BatchLat) * size_t(n),
                                hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + L.items, items.data(), sizeof(int4) * items.size(),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + L.acc, 0, sizeof(Acc) * size_t(n), stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + L.retired, 0, 4 * size_t(n), stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + L.ctl, 0, sizeof(BatchCtl), stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + L.x, 0, L.t - L.x, stream);   // x, xa
  if (e == hipSuccess) e = hipMemsetAsync(base + L.t, 0, L.total - L.t, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return cleanup(set_error(LBM_EHIP, "batch set-up: %s", hipGetErrorString(e)));

  BatchArgs& a = b->args;
  a.lats = reinterpret_cast<const BatchLat*>(base + L.lats);
  a.items = reinterpret_cast<const int4*>(base + L.items);
  a.nlat = n;
  a.nitems = L.nitems;
  a.xper = 0;
  a.yper = yper;
  a.s_e = p->s_e;
  a.s_eps = p->s_eps;
  a.part[0] = reinterpret_cast<float*>(base + L.part0);
  a.part[1] = reinterpret_cast<float*>(base + L.part1);
  a.acc = reinterpret_cast<Acc*>(base + L.acc);
  a.hist = reinterpret_cast<double*>(base + L.hist);
  a.hist_cap = p->history_cap;
  a.retired = reinterpret_cast<int*>(base + L.retired);
  a.ctl = reinterpret_cast<BatchCtl*>(base + L.ctl);
  a.spin_limit = p->spin_limit > 0 ? p->spin_limit : kDefaultSpin;
  a.log_start = p->log_start;
  a.log_every = p->log_every > 0 ? p->log_every : 1;
  a.log_slots = p->log_slots;
  a.log_rows = p->log_rows;
  a.x = reinterpret_cast<float*>(base + L.x);
  a.xa = reinterpret_cast<float*>(base + L.xa);
  a.t = reinterpret_cast<float*>(base + L.t);

  // Co-resident grid of the persistent mode.  A workgroup of 256 threads
  // puts one wave on each of a CU's four SIMDs, so a CU holds k workgroups
  // at once when k waves of the kernel fit one SIMD: k times its VGPRs
  // (allocated in granules of 8 from the 512 of the unified register file)
  // within 512, k <= 8 waves, k times its LDS within the CU's 160 KiB, and
  // k times its SGPRs within the SIMD's 800 (a wave allocates at most 112,
  // so any k <= 7 fits).  The smaller of that bound and the occupancy query
  // is taken; the grid uses groups_per_cu (default kBatchGroupsPerCu) of
  // them per CU.
  int dev = 0, cus = 0, per_cu = 0;
  hipFuncAttributes fa{};
  const void* kfn = p->collision == LBM_MRT ? reinterpret_cast<const void*>(k_batch<1>)
                                            : reinterpret_cast<const void*>(k_batch<0>);
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = p->collision == LBM_MRT
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<1>, kBlock, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<0>, kBlock, 0);
  if (e == hipSuccess) e = hipFuncGetAttributes(&fa, kfn);
  if (e != hipSuccess || per_cu < 1 || cus < 1)
    return cleanup(set_error(LBM_EHIP, "occupancy query failed"));
  const int vgpr = std::max(8, (fa.numRegs + 7) / 8 * 8);
  const int lds = std::max<int>(1, int(fa.sharedSizeBytes));
  const int fit = std::min({512 / vgpr, 8, 7, (160 * 1024) / lds, per_cu});
  const int per = p->groups_per_cu > 0 ? p->groups_per_cu : kBatchGroupsPerCu;
  if (p->launch == LBM_BATCH_PERSISTENT && per > fit)
    return cleanup(set_error(LBM_EINVAL, "groups_per_cu %d exceeds the %d workgroups per CU the "
                             "persistent kernel can hold at once (%d VGPRs, %d B of LDS)",
                             per, fit, fa.numRegs, lds));
  // The item split gives each XCD one eighth of the workgroups: the grid is a
  // multiple of 8, and no larger than the items need.
  const int wanted = (L.nitems + 8 * kWaves - 1) / (8 * kWaves) * 8;
  b->grid = std::max(8, std::min(std::min(per, fit) * cus / 8 * 8, wanted));
  // items of the XCD with the most (whole rounds of chunks)
  const int per_xcd = (L.nitems + 8 * kItemChunk - 1) / (8 * kItemChunk) * kItemChunk;
  b->grid_step = 8 * std::max(1, (per_xcd + kWaves - 1) / kWaves);
  if (getenv("LBM_BATCH_VERBOSE"))
    fprintf(stderr, "lbm_batch: %d CUs, occupancy query %d, resource bound %d workgroups per CU "
            "(%d VGPRs, %d B LDS), grid %d\n", cus, per_cu, fit, fa.numRegs, lds, b->grid);
  b->steps = 0;
  b->fixed_slots = 0;
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (b) (void)hipStreamSynchronize(b->stream);   // a persistent launch may still run
  delete b;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b) return set_error(LBM_EINVAL, "NULL batch");
  if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps < 0");
  if (nsteps == 0) return LBM_OK;
  BatchArgs a = b->args;
  a.step0 = b->steps;
  a.nsteps = nsteps;
  if (b->p.launch == LBM_BATCH_PER_STEP) {
    a.nsteps = 1;
    for (int64_t i = 0; i < nsteps; ++i) {
      a.step0 = b->steps + i;
      if (b->p.collision == LBM_MRT)
        hipLaunchKernelGGL(k_batch_step<1>, dim3(b->grid_step), dim3(kBlock), 0, b->stream, a, int(i > 0));
      else
        hipLaunchKernelGGL(k_batch_step<0>, dim3(b->grid_step), dim3(kBlock), 0, b->stream, a, int(i > 0));
    }
    const int flush_grid = std::max(1, std::min(b->nlat, 1024));
    hipLaunchKernelGGL(k_batch_flush, dim3(flush_grid), dim3(kBlock), 0, b->stream, a,
                       int((b->steps + nsteps - 1) & 1));
    BTRY(hipGetLastError());
    b->steps += nsteps;
    return LBM_OK;
  }
  void* kargs[] = {&a};
  const void* fn = b->p.collision == LBM_MRT ? reinterpret_cast<const void*>(k_batch<1>)
                                             : reinterpret_cast<const void*>(k_batch<0>);
  BTRY(hipLaunchCooperativeKernel(fn, dim3(b->grid), dim3(kBlock), kargs, 0, b->stream));
  b->steps += nsteps;
  return LBM_OK;
}

lbm_status lbm_batch_forces(lbm_batch* b, int32_t l, lbm_force_out* out) {
  if (!b || !out || l < 0 || l >= b->nlat) return set_error(LBM_EINVAL, "bad argument");
  lbm_status st = batch_sync(b);
  if (st) return st;
  Acc a;
  BTRY(hipMemcpy(&a, b->args.acc + l, sizeof a, hipMemcpyDeviceToHost));
  out->fx = a.fx;
  out->fy = a.fy;
  out->fx_sum = a.fx_sum;
  out->fy_sum = a.fy_sum;
  out->mass = a.mass;
  out->step = b->steps;
  out->n_fallback = 0;
  out->nonfinite = a.nonfinite;
  out->reserved = 0;
  if (a.nonfinite) return set_error(LBM_EUNSTABLE, "lattice %d produced a non-finite force or mass", l);
  return LBM_OK;
}

lbm_status lbm_batch_force_history(lbm_batch* b, int32_t l, double* fx, double* fy, int64_t cap,
                                   int64_t* n) {
  if (!b || !n || l < 0 || l >= b->nlat || (cap > 0 && (!fx || !fy)))
    return set_error(LBM_EINVAL, "bad argument");
  lbm_status st = batch_sync(b);
  if (st) return st;
  const int64_t m = std::min(std::min(b->steps, b->p.history_cap), cap);
  *n = std::max<int64_t>(m, 0);
  if (m <= 0) return LBM_OK;
  std::vector<double> h(size_t(m) * 3);
  BTRY(hipMemcpy(h.data(), b->args.hist + int64_t(l) * b->p.history_cap * 3, h.size() * 8,
                 hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < m; ++k) {
    fx[k] = h[3 * k];
    fy[k] = h[3 * k + 1];
  }
  return LBM_OK;
}

lbm_status lbm_batch_read_populations(lbm_batch* b, int32_t l, double* host) {
  if (!b || !host || l < 0 || l >= b->nlat) return set_error(LBM_EINVAL, "bad argument");
  lbm_status st = batch_sync(b);
  if (st) return st;
  const BatchLat& d = b->lat[size_t(l)];
  const int cur = int(b->steps & 1);
  double* stage = reinterpret_cast<double*>(d.buf[cur ^ 1]);    // spare buffer
  const size_t spare = size_t(9) * size_t(d.plane) * 4;
  const int chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(d.ny), spare / (size_t(9) * d.nx * 8))));
  const size_t nx = size_t(d.nx), plane = nx * size_t(d.ny);
  for (int y0 = 0; y0 < d.ny; y0 += chunk) {
    const int rows = std::min(chunk, d.ny - y0);
    const size_t cnt = size_t(rows) * nx;
    BTRY(launch_read(LBM_FP32_OFFSET, d.buf[cur], stage, d.nx, d.pitch, d.plane, y0, rows, b->stream));
    for (int q = 0; q < 9; ++q)
      BTRY(hipMemcpyAsync(host + q * plane + y0 * nx, stage + q * cnt, cnt * 8, hipMemcpyDeviceToHost,
                          b->stream));
    BTRY(hipStreamSynchronize(b->stream));
  }
  // the staging overwrote the spare buffer: restore it (solid nodes are never
  // rewritten by a step)
  BTRY(hipMemcpyAsync(d.buf[cur ^ 1], d.buf[cur], spare, hipMemcpyDeviceToDevice, b->stream));
  BTRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

lbm_status lbm_batch_retired(lbm_batch* b, int32_t* flags) {
  if (!b || !flags) return set_error(LBM_EINVAL, "NULL argument");
  lbm_status st = batch_sync(b);
  if (st) return st;
  BTRY(hipMemcpy(flags, b->args.retired, 4 * size_t(b->nlat), hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_batch_dataset(lbm_batch* b, const float** x, const float** xa, const float** t,
                             int64_t* n) {
  if (!b || !x || !xa || !t || !n) return set_error(LBM_EINVAL, "NULL argument");
  const lbm_batch_params& p = b->p;
  int64_t slots = 0;
  if (p.log_slots > 0 && b->steps > p.log_start)
    slots = std::min(p.log_slots, (b->steps - 1 - p.log_start) / std::max<int64_t>(p.log_every, 1) + 1);
  if (slots > b->fixed_slots) {
    const int64_t n0 = b->fixed_slots * p.log_rows, n1 = slots * p.log_rows;
    hipLaunchKernelGGL(k_fix_targets, dim3(unsigned((n1 - n0 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       b->stream, b->args.t, b->args.x, n0, n1);
    BTRY(hipGetLastError());
    b->fixed_slots = slots;
  }
  lbm_status st = batch_sync(b);
  if (st) return st;
  *x = b->args.x;
  *xa = b->args.xa;
  *t = b->args.t;
  *n = slots * p.log_rows;
  return LBM_OK;
}

}  // extern "C"
