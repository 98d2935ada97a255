// Host side of the C ABI declared in include/lbm.h.
//
// The context borrows a caller-owned device workspace and stream; it carves
// the workspace into the two population buffers, the per-node link words,
// the partial-sum buffers, the FP64 accumulators, the force history and the
// network image, and enqueues the kernels of lbm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "d2q9_dev.hpp"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {
thread_local std::string g_err;
}

namespace lbm {
lbm_status set_error(lbm_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int64_t build_links(const uint8_t* mask, int nx, int ny, int pitch, int nchunk, bool xper,
                    bool yper, uint32_t* links, uint8_t* chunk) {
  int64_t n_fluid = 0;
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      uint32_t w = 0;
      if (mask[int64_t(y) * nx + x]) {
        w = LINK_SOLID;
      } else {
        ++n_fluid;
        if (!xper && x == 0) w |= LINK_INLET;
        if (!xper && x == nx - 1) w |= LINK_OUTLET;
        for (int q = 1; q < 9; ++q) {
          int sx = x - cx(q), sy = y - cy(q);
          if (sx < 0 || sx >= nx) {
            if (!xper) continue;               // unknown: inlet / outlet column
            sx = (sx + nx) % nx;
          }
          if (sy < 0 || sy >= ny) {
            if (!yper) {
              w |= 1u << (LINK_BB_SHIFT + q);  // wall
              continue;
            }
            sy = (sy + ny) % ny;
          }
          const uint8_t m = mask[int64_t(sy) * nx + sx];
          if (m) w |= 1u << (LINK_BB_SHIFT + q);
          if (m == 1) w |= 1u << (LINK_FORCE_SHIFT + q);
        }
      }
      links[size_t(y) * pitch + x] = w;
      if (w) chunk[size_t(y) * nchunk + (x / kChunk)] = 1;
    }
  }
  return n_fluid;
}

}  // namespace lbm

namespace {

#define fail lbm::set_error

lbm_status hip_fail(hipError_t e, const char* what) {
  return fail(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int precision) {
  return precision == LBM_FP64 ? 8 : (precision == LBM_FP32_OFFSET ? 4 : 2);
}

// Bulk path: the vector tile pays off once the grid holds many waves per
// resident slot (large lattices); small lattices use the scalar tile.
// params.bulk_path may force either.
constexpr int64_t kVectorPathMinNodes = int64_t(12) << 20;

int choose_path(const lbm_params& p) {
  if (p.bulk_path == LBM_PATH_SCALAR) return PATH_SCALAR;
  if (p.bulk_path == LBM_PATH_VECTOR) return PATH_VECTOR;
  return int64_t(p.nx) * p.ny >= kVectorPathMinNodes ? PATH_VECTOR : PATH_SCALAR;
}

struct Layout {
  int path;
  int pitch, nchunk, rows, ntx, nty, nn_max, nslots_max;
  int64_t plane;
  size_t A, B, links, chunk, inlet, part0, part1, lvl0, lvl1, acc, hist, mlp, cbc, cbc_dt, total;
};

// Bulk tiles per chunk dealt to the XCDs in turn, or 0 for one band per XCD.
// Bands are kept where each XCD's band covers a whole number of MiB of every
// population plane (4096 x 1024 FP32: 128 rows, 2 MiB, 0.5 % ahead of
// chunks; 2048 x 1024 and 4096 x 512: 1 MiB, 0.6-0.8 % ahead); elsewhere
// chunks of about 512 KiB of a plane, measured 8-16 % faster than bands at
// 4096 x 896, 4096 x 1280, 3584 x 1024 and 6144 x 1024 (bands then put the
// XCDs' concurrent rows at spacings that load the HBM channels unevenly).
int xcd_chunk_tiles(const Layout& lay, int precision) {
  const int64_t tile_row = int64_t(lay.pitch) * lay.rows * int64_t(elem_size(precision));
  const int64_t band = lay.nty / 8 * tile_row;
  if (lay.nty % 8 == 0 && band % (int64_t(1) << 20) == 0) return 0;
  const int64_t rows = std::max<int64_t>(1, ((int64_t(512) << 10) + tile_row / 2) / tile_row);
  return int(rows) * lay.ntx;
}

#ifndef LBM_PLANE_RESIDUE
#define LBM_PLANE_RESIDUE 4352
#endif
// Elements per population plane: ny x pitch, padded so that the plane's
// byte stride lies kPlaneResidue bytes past a multiple of 64 KiB.  Unpadded
// power-of-two planes (4096 x 1024 FP32: 16 MiB) send the nine populations
// of a row to the same HBM channels; the two-step kernel then ran 5 % slower
// (88.2 against 83.9 thousand MLUPS; a 256-byte residue gave 86.3).
constexpr int64_t kPlaneResidue = LBM_PLANE_RESIDUE;
int64_t padded_plane(int64_t nodes, size_t es) {
  if (kPlaneResidue < 0) return nodes;
  const int64_t bytes = nodes * int64_t(es);
  const int64_t pad = ((kPlaneResidue - bytes % 65536) % 65536 + 65536) % 65536;
  return (bytes + pad) / int64_t(es);
}

Layout make_layout(const lbm_params& p) {
  Layout L{};
  L.path = choose_path(p);
  L.pitch = int(align_up(size_t(p.nx), kChunk));   // whole tiles per row
  L.nchunk = L.pitch / kChunk;
  L.rows = tile_rows(L.path);
  L.ntx = L.nchunk;
  L.nty = (p.ny + L.rows - 1) / L.rows;
  L.nn_max = (p.ny + kNnRows - 1) / kNnRows;
  L.nslots_max = (L.nn_max + 8 + L.ntx * L.nty) * kWaves;   // + padding to a multiple of 8
  // two-step launches write two steps' slots (outlet blocks included),
  // three-step launches three steps' slots
  const int row_bytes = L.pitch * int(elem_size(p.precision));
  L.nslots_max = std::max(L.nslots_max,
                          2 * (pair_waves(p.nx, p.ny, pair_rows(p.nx, p.ny, row_bytes)) +
                               pair_outlet_blocks(p.ny) * kWaves));
  if (tri_supported(p.precision))
    L.nslots_max = std::max(L.nslots_max, 3 * (tri_waves(p.nx, p.ny, tri_rows(p.nx, p.ny, row_bytes, 0)) +
                                               tri_outlet_blocks(p.ny, true) * kWaves));
  L.plane = padded_plane(int64_t(p.ny) * L.pitch, elem_size(p.precision));
  const size_t pop = size_t(9) * size_t(L.plane) * elem_size(p.precision);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.A = take(pop);
  L.B = take(pop);
  L.links = take(size_t(p.ny) * L.pitch * 4);
  L.chunk = take(size_t(p.ny) * L.nchunk);
  L.inlet = take(size_t(p.ny) * 8);
  L.part0 = take(size_t(L.nslots_max) * kPartials * 8);   // one slot per wave
  L.part1 = take(size_t(L.nslots_max) * kPartials * 8);
  L.lvl0 = take(size_t(3 * kReducers) * 4 * 8);   // the sums of up to three steps per launch
  L.lvl1 = take(size_t(3 * kReducers) * 4 * 8);
  L.acc = take(sizeof(Acc));
  L.hist = take(size_t(std::max<int64_t>(p.history_cap, 0)) * 3 * 8);
  L.mlp = take(sizeof(MlpDev));
  L.cbc = take(sizeof(CbcDev));
  L.cbc_dt = take(size_t(2) * p.ny * 4 * 8);    // two buffers: two-step launches swap them
  L.total = o;
  return L;
}

lbm_status check_params(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 8 || p->ny < 8) return fail(LBM_EINVAL, "nx, ny must be >= 8 (got %d, %d)", p->nx, p->ny);
  // one population plane (with its padding) must stay below 4 GiB (32-bit
  // byte offsets)
  if ((int64_t(p->nx) + 255) * p->ny * 8 + 65536 >= (int64_t(1) << 32))
    return fail(LBM_EINVAL, "lattice too large (%d x %d)", p->nx, p->ny);
  if (p->precision < LBM_FP64 || p->precision > LBM_FP16_OFFSET)
    return fail(LBM_EINVAL, "bad precision %d", p->precision);
  if (p->collision != LBM_BGK && p->collision != LBM_MRT)
    return fail(LBM_EINVAL, "bad collision %d", p->collision);
  if (p->lateral != LBM_LATERAL_WALLS && p->lateral != LBM_LATERAL_PERIODIC)
    return fail(LBM_EINVAL, "bad lateral %d", p->lateral);
  if (p->xbc != LBM_X_INOUT && p->xbc != LBM_X_PERIODIC) return fail(LBM_EINVAL, "bad xbc %d", p->xbc);
  if (p->launch < LBM_LAUNCH_AUTO || p->launch > LBM_LAUNCH_TRIPLES_HELD)
    return fail(LBM_EINVAL, "bad launch %d", p->launch);
  if ((p->launch == LBM_LAUNCH_TRIPLES || p->launch == LBM_LAUNCH_TRIPLES_PLAIN ||
       p->launch == LBM_LAUNCH_TRIPLES_HELD) && !tri_supported(p->precision))
    return fail(LBM_EINVAL, "three-step launches need LBM_FP32_OFFSET or LBM_FP16_OFFSET");
  if ((p->launch == LBM_LAUNCH_PAIRS_HELD || p->launch == LBM_LAUNCH_TRIPLES_HELD) &&
      p->precision == LBM_FP16_OFFSET)
    return fail(LBM_EINVAL, "the held walk needs LBM_FP64 or LBM_FP32_OFFSET");
  if (p->bulk_path < LBM_PATH_AUTO || p->bulk_path > LBM_PATH_VECTOR)
    return fail(LBM_EINVAL, "bad bulk_path %d", p->bulk_path);
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be > 0.5 (got %g)", p->tau);
  if (!std::isfinite(p->u_in) || std::fabs(p->u_in) >= 0.5)
    return fail(LBM_EINVAL, "|u_in| must be < 0.5 (got %g)", p->u_in);
  if (!(p->rho_out > 0)) return fail(LBM_EINVAL, "rho_out must be > 0");
  if (p->history_cap < 0) return fail(LBM_EINVAL, "history_cap must be >= 0");
  return LBM_OK;
}

uint16_t bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

}  // namespace

struct lbm_ctx {
  lbm_params p;
  Layout lay;
  hipStream_t stream;
  char* ws;
  void* buf[2];
  int cur;          // buf[cur] holds the post-collision state
  void* part[2];
  double* lvl[2];
  int pcur;         // part[pcur] and lvl[pcur] are written by the next step
  bool pend1;       // part[pcur ^ 1] holds the slots of the previous step
  bool pend2;       // lvl[pcur ^ 1] holds the level-1 sums of the step before
  bool geometry;
  bool has_profile;
  int outflow;
  int n_nn;
  double n_fluid;
  int64_t steps;

  uint32_t* links() { return reinterpret_cast<uint32_t*>(ws + lay.links); }
  uint8_t* chunk() { return reinterpret_cast<uint8_t*>(ws + lay.chunk); }
  double* inlet() { return reinterpret_cast<double*>(ws + lay.inlet); }
  Acc* acc() { return reinterpret_cast<Acc*>(ws + lay.acc); }
  double* hist() { return reinterpret_cast<double*>(ws + lay.hist); }
  MlpDev* mlp() { return reinterpret_cast<MlpDev*>(ws + lay.mlp); }
  CbcDev* cbc() { return reinterpret_cast<CbcDev*>(ws + lay.cbc); }
  int dtcur;        // cbc_dt(dtcur) holds the outlet time derivatives
  double* cbc_dt(int i = -1) {
    return reinterpret_cast<double*>(ws + lay.cbc_dt) + size_t(i < 0 ? dtcur : i) * p.ny * 4;
  }
  size_t pop_bytes() const { return size_t(9) * size_t(lay.plane) * elem_size(p.precision); }

  StepLaunch launch() {
    StepLaunch L{};
    L.precision = p.precision;
    L.collision = p.collision;
    L.path = lay.path;
    L.A = buf[cur];
    L.B = buf[cur ^ 1];
    L.links = links();
    L.chunk = chunk();
    L.inlet = has_profile ? inlet() : nullptr;
    L.part_w = part[pcur];
    L.part_r = part[pcur ^ 1];
    L.lvl_w = lvl[pcur];
    L.lvl_r = lvl[pcur ^ 1];
    L.reduce1 = pend1;
    L.reduce2 = pend2;
    L.acc = acc();
    L.hist = hist();
    L.hist_cap = p.history_cap;
    L.mlp = mlp();
    L.cbc = cbc();
    L.cbc_dt = cbc_dt();
    L.cbc_dt_w = cbc_dt(dtcur ^ 1);
    L.outlet = outflow == LBM_OUT_CBC ? OUTLET_CBC : OUTLET_NN;
    L.nx = p.nx;
    L.ny = p.ny;
    L.pitch = lay.pitch;
    L.nchunk = lay.nchunk;
    L.plane = lay.plane;
    L.rows = lay.rows;
    L.ntx = lay.ntx;
    L.nty = lay.nty;
    L.n_nn = n_nn;
    L.nspecial = (1 + kReducers + n_nn + 7) / 8 * 8;
    L.nblocks = L.nspecial + lay.ntx * lay.nty;
    L.xcd_chunk = xcd_chunk_tiles(lay, p.precision);
    // two-step launches: with the neural outlet its blocks take the last
    // columns and come first; the strips take the other columns
    L.pair_out = n_nn ? pair_outlet_blocks(p.ny) : 0;
    L.pair_nx = L.pair_out ? p.nx - pair_outlet_cols() : p.nx;
    L.pair_rows = pair_rows(p.nx, p.ny, lay.pitch * int(elem_size(p.precision)));
    L.pair_hold = p.launch == LBM_LAUNCH_PAIRS_HELD    ? 1
                  : p.launch == LBM_LAUNCH_PAIRS_PLAIN ? 0
                                                       : pair_hold(p.precision, 9 * lay.plane * int64_t(elem_size(p.precision)));
    L.pair_nslots = pair_waves(L.pair_nx, p.ny, L.pair_rows) + L.pair_out * kWaves;
    L.pair_chunk = pair_chunk(L.pair_nx);
    // three-step launches: the neural or characteristic outlet's blocks take
    // the last columns and come first
    L.tri_out = outflow == LBM_OUT_ZOUHE ? 0 : tri_outlet_blocks(p.ny, outflow == LBM_OUT_CBC);
    L.tri_nx = L.tri_out ? p.nx - pair_outlet_cols() : p.nx;
    L.tri_rows = tri_rows(L.tri_nx, p.ny, lay.pitch * int(elem_size(p.precision)), L.tri_out);
    L.tri_nslots = tri_waves(L.tri_nx, p.ny, L.tri_rows) + L.tri_out * kWaves;
    L.tri_chunk = tri_chunk(L.tri_nx);
    L.tri_hold = p.launch == LBM_LAUNCH_TRIPLES_HELD    ? 1
                 : p.launch == LBM_LAUNCH_TRIPLES_PLAIN ? 0
                                                        : pair_hold(p.precision, 9 * lay.plane * int64_t(elem_size(p.precision)));
    L.nslots = (L.nspecial - 1 - kReducers + lay.ntx * lay.nty) * kWaves;
    L.xper = p.xbc == LBM_X_PERIODIC;
    L.yper = p.lateral == LBM_LATERAL_PERIODIC;
    L.omega = 1.0 / p.tau;
    L.s_e = p.s_e;
    L.s_eps = p.s_eps;
    L.s_q = p.s_q > 0 ? p.s_q : 1.0 / (0.5 + (3.0 / 16.0) / (p.tau - 0.5));
    L.u_in = p.u_in;
    L.one_minus_rho_out = 1.0 - p.rho_out;
    L.n_fluid = n_fluid;
    return L;
  }

  // rows of a staging chunk of `per_node` doubles per node that fit in the
  // spare population buffer
  int stage_rows(int per_node) const {
    const size_t bytes = pop_bytes();
    const size_t row = size_t(per_node) * size_t(p.nx) * 8;
    return int(std::max<size_t>(1, std::min<size_t>(size_t(p.ny), bytes / row)));
  }
};

namespace {

lbm_status reset_counters(lbm_ctx* c) {
  HIP_TRY(hipMemsetAsync(c->acc(), 0, sizeof(Acc), c->stream));
  HIP_TRY(hipMemsetAsync(c->cbc_dt(0), 0, size_t(2) * c->p.ny * 4 * 8, c->stream));
  c->steps = 0;
  c->pend1 = c->pend2 = false;
  c->pcur = 0;
  return LBM_OK;
}

// A was just written; give B the same content (solid nodes are never
// rewritten by a step, so both buffers must hold them).
lbm_status mirror_state(lbm_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->buf[c->cur ^ 1], c->buf[c->cur], c->pop_bytes(),
                         hipMemcpyDeviceToDevice, c->stream));
  return LBM_OK;
}

lbm_status init_state(lbm_ctx* c, const double* rho, const double* ux, const double* uy) {
  InitLaunch I{};
  I.precision = c->p.precision;
  I.A = c->buf[c->cur];
  I.B = c->buf[c->cur ^ 1];
  I.links = c->links();
  I.nx = c->p.nx;
  I.ny = c->p.ny;
  I.pitch = c->lay.pitch;
  I.plane = c->lay.plane;
  I.u_in = c->p.u_in;
  I.noise_amp = c->p.noise_amp;
  I.seed = c->p.seed;
  if (!rho) {
    I.y0 = 0;
    I.rows = c->p.ny;
    I.fields = nullptr;
    HIP_TRY(launch_init(I, c->stream));
    return LBM_OK;
  }
  // host fields are staged through the spare buffer, which the init kernel
  // does not write; the state is mirrored afterwards
  double* stage = static_cast<double*>(c->buf[c->cur ^ 1]);
  I.B = c->buf[c->cur];
  const int chunk = c->stage_rows(3);
  const size_t nx = size_t(c->p.nx);
  for (int y0 = 0; y0 < c->p.ny; y0 += chunk) {
    const int rows = std::min(chunk, c->p.ny - y0);
    const size_t n = size_t(rows) * nx;
    HIP_TRY(hipMemcpyAsync(stage, rho + y0 * nx, n * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(stage + n, ux + y0 * nx, n * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(stage + 2 * n, uy + y0 * nx, n * 8, hipMemcpyHostToDevice, c->stream));
    I.y0 = y0;
    I.rows = rows;
    I.fields = stage;
    HIP_TRY(launch_init(I, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));   // the stage is reused
  }
  return mirror_state(c);
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (check_params(p) != LBM_OK) return 0;
  return make_layout(*p).total;
}

lbm_status lbm_create(const lbm_params* p, void* dev_workspace, size_t bytes, lbm_ctx** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status st = check_params(p);
  if (st) return st;
  if (!dev_workspace) return fail(LBM_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
    return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  const Layout lay = make_layout(*p);
  if (bytes < lay.total)
    return fail(LBM_ENOSPACE, "workspace has %zu bytes, needs %zu", bytes, lay.total);
  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->lay = lay;
  c->stream = static_cast<hipStream_t>(p->stream);
  c->ws = static_cast<char*>(dev_workspace);
  c->buf[0] = c->ws + lay.A;
  c->buf[1] = c->ws + lay.B;
  c->part[0] = c->ws + lay.part0;
  c->part[1] = c->ws + lay.part1;
  c->lvl[0] = reinterpret_cast<double*>(c->ws + lay.lvl0);
  c->lvl[1] = reinterpret_cast<double*>(c->ws + lay.lvl1);
  c->cur = 0;
  c->dtcur = 0;
  c->outflow = LBM_OUT_ZOUHE;
  c->n_nn = 0;
  *out = c;
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c) {
  if (c) (void)hipStreamSynchronize(c->stream);   // queued steps finish first
  delete c;
  return LBM_OK;
}

lbm_status lbm_set_geometry(lbm_ctx* c, const uint8_t* mask) {
  if (!c || !mask) return fail(LBM_EINVAL, "NULL argument");
  const int nx = c->p.nx, ny = c->p.ny, pitch = c->lay.pitch, nch = c->lay.nchunk;
  const bool xper = c->p.xbc == LBM_X_PERIODIC, yper = c->p.lateral == LBM_LATERAL_PERIODIC;
  for (int64_t i = 0; i < int64_t(nx) * ny; ++i)
    if (mask[i] > 2) return fail(LBM_EINVAL, "mask value %d at node %lld", mask[i], (long long)i);
  if (!xper)
    for (int y = 0; y < ny; ++y)
      if (mask[int64_t(y) * nx] || mask[int64_t(y) * nx + nx - 1])
        return fail(LBM_EINVAL, "columns 0 and nx-1 must be fluid (row %d)", y);
  std::vector<uint32_t> links(size_t(ny) * pitch, 0u);
  std::vector<uint8_t> chunk(size_t(ny) * nch, 0);
  const int64_t n_fluid = build_links(mask, nx, ny, pitch, nch, xper, yper, links.data(), chunk.data());
  HIP_TRY(hipMemcpyAsync(c->links(), links.data(), links.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->chunk(), chunk.data(), chunk.size(), hipMemcpyHostToDevice, c->stream));
  c->n_fluid = double(n_fluid);
  lbm_status st = init_state(c, nullptr, nullptr, nullptr);
  if (st) return st;
  st = reset_counters(c);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));     // host vectors go out of scope
  c->geometry = true;
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy) {
  if (!c || !rho || !ux || !uy) return fail(LBM_EINVAL, "NULL argument");
  if (!c->geometry) return fail(LBM_ESTATE, "lbm_set_geometry first");
  lbm_status st = init_state(c, rho, ux, uy);
  if (st) return st;
  return reset_counters(c);
}

lbm_status lbm_set_inlet_profile(lbm_ctx* c, const double* ux) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (!ux) {
    c->has_profile = false;
    return LBM_OK;
  }
  for (int y = 0; y < c->p.ny; ++y)
    if (!std::isfinite(ux[y]) || std::fabs(ux[y]) >= 0.5)
      return fail(LBM_EINVAL, "inlet velocity %g at row %d", ux[y], y);
  HIP_TRY(hipMemcpyAsync(c->inlet(), ux, size_t(c->p.ny) * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->has_profile = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (!c->geometry) return fail(LBM_ESTATE, "lbm_step before lbm_set_geometry");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  if (nsteps == 0) return LBM_OK;
  int64_t s = 0;
  // With params.launch = LBM_LAUNCH_AUTO or LBM_LAUNCH_TRIPLES and FP32 or
  // FP16 offsets, three steps run in each launch (any outflow); the rest of
  // the count as below.
  const bool triples = (c->p.launch == LBM_LAUNCH_AUTO || c->p.launch == LBM_LAUNCH_TRIPLES ||
                        c->p.launch == LBM_LAUNCH_TRIPLES_PLAIN || c->p.launch == LBM_LAUNCH_TRIPLES_HELD) &&
                       tri_supported(c->p.precision);
  if (nsteps >= 3 && triples) {
    for (; s + 2 < nsteps; s += 3) {
      const StepLaunch L = c->launch();
      HIP_TRY(launch_triple(L, c->stream));
      c->pend2 = c->pend1;
      c->pend1 = true;
      c->pcur ^= 1;
      c->cur ^= 1;
      if (c->outflow == LBM_OUT_CBC) c->dtcur ^= 1;    // the launch wrote the other buffer
    }
    StepLaunch F = c->launch();
    HIP_TRY(launch_finalize_triple(F, c->stream));
    c->pend1 = c->pend2 = false;
  }
  // With params.launch other than LBM_LAUNCH_SINGLE, pairs of steps run in
  // one launch each (the same node arithmetic) whatever the outflow.
  if (nsteps - s >= 2 && c->p.launch != LBM_LAUNCH_SINGLE) {
    for (; s + 1 < nsteps; s += 2) {
      const StepLaunch L = c->launch();
      HIP_TRY(launch_pair(L, c->stream));
      c->pend2 = c->pend1;
      c->pend1 = true;
      c->pcur ^= 1;
      c->cur ^= 1;
      if (c->outflow == LBM_OUT_CBC) c->dtcur ^= 1;    // the launch wrote the other buffer
    }
    StepLaunch F = c->launch();
    HIP_TRY(launch_finalize_pair(F, c->stream));
    c->pend1 = c->pend2 = false;
  }
  if (s < nsteps) {
    for (; s < nsteps; ++s) {
      const StepLaunch L = c->launch();
      HIP_TRY(launch_step(L, c->stream));
      c->pend2 = c->pend1;
      c->pend1 = true;
      c->pcur ^= 1;
      c->cur ^= 1;
    }
    StepLaunch F = c->launch();
    HIP_TRY(launch_finalize(F, c->stream));
    c->pend1 = c->pend2 = false;
  }
  c->steps += nsteps;
  return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_forces(lbm_ctx* c, lbm_force_out* out) {
  if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
  Acc a;
  HIP_TRY(hipMemcpyAsync(&a, c->acc(), sizeof a, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  out->fx = a.fx;
  out->fy = a.fy;
  out->fx_sum = a.fx_sum;
  out->fy_sum = a.fy_sum;
  out->mass = a.mass;
  out->step = c->steps;
  out->n_fallback = int64_t(std::llround(a.fallback));
  out->nonfinite = a.nonfinite;
  out->reserved = 0;
  if (a.nonfinite) return fail(LBM_EUNSTABLE, "non-finite force or mass after step %lld", (long long)c->steps);
  return LBM_OK;
}

lbm_status lbm_force_history(lbm_ctx* c, double* fx, double* fy, int64_t cap, int64_t* n) {
  if (!c || !n || (cap > 0 && (!fx || !fy))) return fail(LBM_EINVAL, "NULL argument");
  const int64_t m = std::min(std::min(c->steps, c->p.history_cap), cap);
  *n = std::max<int64_t>(m, 0);
  if (m <= 0) return LBM_OK;
  std::vector<double> h(size_t(m) * 3);
  HIP_TRY(hipMemcpyAsync(h.data(), c->hist(), h.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int64_t t = 0; t < m; ++t) {
    fx[t] = h[3 * t];
    fy[t] = h[3 * t + 1];
  }
  return LBM_OK;
}

lbm_status lbm_set_outflow_model(lbm_ctx* c, int32_t kind, const lbm_mlp* w) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (kind == LBM_OUT_ZOUHE) {
    c->outflow = kind;
    c->n_nn = 0;
    return LBM_OK;
  }
  if (kind != LBM_OUT_NN) return fail(LBM_EINVAL, "bad outflow kind %d", kind);
  if (c->p.xbc != LBM_X_INOUT) return fail(LBM_EINVAL, "neural outflow needs LBM_X_INOUT");
  if (!w) return fail(LBM_EINVAL, "weights are NULL");
  const int ni = w->n_in, h1 = w->n_h1, h2 = w->n_h2;
  if (ni < 1 || ni > 27 || h1 < 1 || h1 > 64 || h2 < 1 || h2 > 64 || w->n_out != 3)
    return fail(LBM_EINVAL, "network must be at most 27-64-64-3 with 3 outputs (got %d-%d-%d-%d)",
                ni, h1, h2, w->n_out);
  if (!w->w1 || !w->b1 || !w->w2 || !w->b2 || !w->w3 || !w->b3 || !w->mu_in || !w->sd_in ||
      !w->mu_out || !w->sd_out)
    return fail(LBM_EINVAL, "a weight array is NULL");
  // A smaller network is embedded in the 27-64-64-3 one: zero weights and
  // biases in the missing places make the extra hidden units exactly 0 and
  // the extra inputs contribute exactly 0.
  MlpDev* h = new MlpDev();
  memset(h, 0, sizeof *h);
  for (int o = 0; o < h1; ++o)
    for (int i = 0; i < ni; ++i) h->w1[o * 32 + i] = bf16_bits(w->w1[o * ni + i]);
  for (int o = 0; o < h2; ++o)
    for (int i = 0; i < h1; ++i) h->w2[o * 64 + i] = bf16_bits(w->w2[o * h1 + i]);
  for (int o = 0; o < 3; ++o)
    for (int i = 0; i < h2; ++i) h->w3[o * 64 + i] = bf16_bits(w->w3[o * h2 + i]);
  for (int o = 0; o < h1; ++o) h->b1[o] = w->b1[o];
  for (int o = 0; o < h2; ++o) h->b2[o] = w->b2[o];
  for (int o = 0; o < 3; ++o) {
    h->b3[o] = w->b3[o];
    h->mu_out[o] = w->mu_out[o];
    h->sd_out[o] = w->sd_out[o];
  }
  for (int i = 0; i < 27; ++i) {
    h->mu_in[i] = i < ni ? w->mu_in[i] : 0.0f;
    h->inv_sd_in[i] = i < ni ? 1.0f / w->sd_in[i] : 1.0f;
  }
  h->mass_bound = float(w->mass_bound);
  hipError_t e = hipMemcpyAsync(c->mlp(), h, sizeof *h, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  delete h;
  if (e != hipSuccess) return hip_fail(e, "upload of the network");
  c->outflow = kind;
  c->n_nn = c->lay.nn_max;
  return LBM_OK;
}

lbm_status lbm_set_outflow_cbc(lbm_ctx* c, const lbm_cbc* p) {
  if (!c || !p) return fail(LBM_EINVAL, "NULL argument");
  if (c->p.xbc != LBM_X_INOUT) return fail(LBM_EINVAL, "characteristic outflow needs LBM_X_INOUT");
  if (c->p.lateral != LBM_LATERAL_PERIODIC)
    return fail(LBM_EINVAL, "characteristic outflow needs periodic laterals (no corner treatment "
                "where the outlet meets a wall)");
  if (!std::isfinite(p->sigma) || !std::isfinite(p->kappa2) || !(p->mach >= 0 && p->mach < 1) ||
      !(p->length > 0) || !std::isfinite(p->length) || !(p->rho_inf > 0) || !std::isfinite(p->rho_inf))
    return fail(LBM_EINVAL, "bad characteristic outflow parameters (sigma %g, kappa2 %g, mach %g, "
                "length %g, rho_inf %g)", p->sigma, p->kappa2, p->mach, p->length, p->rho_inf);
  CbcDev h;
  memset(&h, 0, sizeof h);
  h.sigma = p->sigma;
  h.kappa2 = p->kappa2;
  h.kappa1_coef = (1.0 - p->mach * p->mach) * std::sqrt(1.0 / 3.0) / p->length;
  h.rho_inf_m1 = p->rho_inf - 1.0;
  if (const lbm_cbc_net* n = p->net) {
    if (!n->w1 || !n->b1 || !n->w2 || !n->b2 || !n->w3 || !n->b3 || !n->mu_in || !n->sd_in)
      return fail(LBM_EINVAL, "a tuning network array is NULL");
    for (int i = 0; i < kCbcIn; ++i)
      if (!(n->sd_in[i] > 0)) return fail(LBM_EINVAL, "sd_in[%d] must be > 0", i);
    if (!std::isfinite(n->leaky_slope) || !std::isfinite(n->sigma_scale) ||
        !std::isfinite(n->sigma_shift) || !std::isfinite(n->kappa_scale) ||
        !std::isfinite(n->kappa_shift))
      return fail(LBM_EINVAL, "bad tuning network output maps");
    memcpy(h.w1, n->w1, sizeof h.w1);
    memcpy(h.b1, n->b1, sizeof h.b1);
    memcpy(h.w2, n->w2, sizeof h.w2);
    memcpy(h.b2, n->b2, sizeof h.b2);
    memcpy(h.w3, n->w3, sizeof h.w3);
    memcpy(h.b3, n->b3, sizeof h.b3);
    memcpy(h.mu_in, n->mu_in, sizeof h.mu_in);
    memcpy(h.sd_in, n->sd_in, sizeof h.sd_in);
    h.leaky = n->leaky_slope;
    h.sigma_scale = n->sigma_scale;
    h.sigma_shift = n->sigma_shift;
    h.kappa_scale = n->kappa_scale;
    h.kappa_shift = n->kappa_shift;
    h.has_net = 1;
  }
  HIP_TRY(hipMemcpyAsync(c->cbc(), &h, sizeof h, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->cbc_dt(0), 0, size_t(2) * c->p.ny * 4 * 8, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->outflow = LBM_OUT_CBC;
  c->n_nn = c->lay.nn_max;
  return LBM_OK;
}

lbm_status lbm_mlp_forward(lbm_ctx* c, const float* x, float* s, int64_t n) {
  if (!c || (n > 0 && (!x || !s))) return fail(LBM_EINVAL, "NULL argument");
  if (c->outflow != LBM_OUT_NN) return fail(LBM_ESTATE, "no network set");
  if (n < 0) return fail(LBM_EINVAL, "n < 0");
  HIP_TRY(launch_mlp_forward(c->mlp(), x, s, n, c->stream));
  return LBM_OK;
}

lbm_status lbm_read_populations(lbm_ctx* c, double* host) {
  if (!c || !host) return fail(LBM_EINVAL, "NULL argument");
  if (!c->geometry) return fail(LBM_ESTATE, "lbm_set_geometry first");
  double* stage = static_cast<double*>(c->buf[c->cur ^ 1]);
  const int chunk = c->stage_rows(9);
  const size_t nx = size_t(c->p.nx), plane = nx * size_t(c->p.ny);
  for (int y0 = 0; y0 < c->p.ny; y0 += chunk) {
    const int rows = std::min(chunk, c->p.ny - y0);
    const size_t n = size_t(rows) * nx;
    HIP_TRY(launch_read(c->p.precision, c->buf[c->cur], stage, c->p.nx, c->lay.pitch, c->lay.plane,
                        y0, rows, c->stream));
    for (int q = 0; q < 9; ++q)
      HIP_TRY(hipMemcpyAsync(host + q * plane + y0 * nx, stage + q * n, n * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  // the staging overwrote the spare buffer: restore it, since its solid nodes
  // are never rewritten by a step
  lbm_status st = mirror_state(c);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_read_macroscopic(lbm_ctx* c, double* rho, double* ux, double* uy) {
  if (!c || !rho || !ux || !uy) return fail(LBM_EINVAL, "NULL argument");
  if (!c->geometry) return fail(LBM_ESTATE, "lbm_set_geometry first");
  double* stage = static_cast<double*>(c->buf[c->cur ^ 1]);
  const int chunk = c->stage_rows(3);
  const size_t nx = size_t(c->p.nx);
  double* out[3] = {rho, ux, uy};
  for (int y0 = 0; y0 < c->p.ny; y0 += chunk) {
    const int rows = std::min(chunk, c->p.ny - y0);
    const size_t n = size_t(rows) * nx;
    HIP_TRY(launch_macro(c->p.precision, c->buf[c->cur], stage, c->p.nx, c->lay.pitch, c->lay.plane,
                         y0, rows, c->stream));
    for (int k = 0; k < 3; ++k)
      HIP_TRY(hipMemcpyAsync(out[k] + y0 * nx, stage + k * n, n * 8, hipMemcpyDeviceToHost,
                             c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  // the staging overwrote the spare buffer, whose solid nodes a step never
  // rewrites: restore it
  lbm_status st = mirror_state(c);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_write_populations(lbm_ctx* c, const double* host) {
  if (!c || !host) return fail(LBM_EINVAL, "NULL argument");
  if (!c->geometry) return fail(LBM_ESTATE, "lbm_set_geometry first");
  double* stage = static_cast<double*>(c->buf[c->cur ^ 1]);
  const int chunk = c->stage_rows(9);
  const size_t nx = size_t(c->p.nx), plane = nx * size_t(c->p.ny);
  for (int y0 = 0; y0 < c->p.ny; y0 += chunk) {
    const int rows = std::min(chunk, c->p.ny - y0);
    const size_t n = size_t(rows) * nx;
    for (int q = 0; q < 9; ++q)
      HIP_TRY(hipMemcpyAsync(stage + q * n, host + q * plane + y0 * nx, n * 8,
                             hipMemcpyHostToDevice, c->stream));
    // the write-back kernel targets A twice (its B argument is A as well)
    HIP_TRY(launch_write(c->p.precision, c->buf[c->cur], c->buf[c->cur], stage, c->p.nx,
                         c->lay.pitch, c->lay.plane, y0, rows, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return mirror_state(c);
}

}  // extern "C"
