// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {

// Two shapes of bulk tile, chosen per lattice when the context is created:
//   scalar (PATH_SCALAR): one node per thread, a workgroup covers 256 columns
//     of one row, each pull is a (possibly misaligned) 4-byte load;
//   vector (PATH_VECTOR): kVec = 4 consecutive nodes per lane, one row per
//     wave, four rows per workgroup, aligned 16-byte loads and a cross-lane
//     shift for the +-1 columns.
// Both cover kChunk = 256 columns per row.
enum { PATH_SCALAR = 0, PATH_VECTOR = 1 };
constexpr int kBlock = 256;                          // threads per workgroup
constexpr int kVec = 4;
constexpr int kChunk = 256;                          // x-extent of a bulk tile
constexpr int tile_rows(int path) { return path == PATH_SCALAR ? 1 : kBlock / 64; }
constexpr int kNnRows = 64;        // outlet rows handled by one neural block
constexpr int kPartials = 4;       // fx, fy, sum of (rho - 1), fallback count
constexpr int kWaves = kBlock / 64;
constexpr int kReducers = 32;      // workgroups reducing the previous step's partials

// Accumulators written only by the reducing workgroup (fixed-order FP64).
struct Acc {
  double fx, fy, fx_sum, fy_sum, mass;
  double fallback;
  int64_t n_reduced;
  int32_t nonfinite;
  int32_t pad;
};

// Device image of the outflow MLP: BF16 weights padded for 16x16x32 MFMA
// tiles, FP32 biases and affine maps.
struct MlpDev {
  uint16_t w1[64 * 32];   // [out][in], in padded 27 -> 32 with zeros
  uint16_t w2[64 * 64];   // [out][in]
  uint16_t w3[16 * 64];   // [out][in], out padded 3 -> 16 with zeros
  float b1[64], b2[64], b3[16];
  float mu_in[32], inv_sd_in[32];   // padded entries: mu 0, inv 0
  float mu_out[4], sd_out[4];
  float mass_bound;
  float pad[3];
};

// Device image of the characteristic outflow (Sec. 4): fixed sigma,
// kappa_2, or the 9-20-20-2 tuning network with its output maps.
constexpr int kCbcIn = 9, kCbcHidden = 20;
struct CbcDev {
  float w1[kCbcHidden * kCbcIn], b1[kCbcHidden];
  float w2[kCbcHidden * kCbcHidden], b2[kCbcHidden];
  float w3[2 * kCbcHidden], b3[2];
  float mu_in[kCbcIn], sd_in[kCbcIn];
  int has_net;
  int pad;
  double leaky, sigma_scale, sigma_shift, kappa_scale, kappa_shift;
  double sigma, kappa2;
  double kappa1_coef;       // (1 - M^2) c_s / L: kappa_1 = sigma * kappa1_coef
  double rho_inf_m1;        // rho_inf - 1
};

// Outflow of the special outlet blocks of the step kernel.
enum { OUTLET_NN = 1, OUTLET_CBC = 2 };

// Reduction pipeline: step t writes one partial slot per wave (part_w); the
// kReducers reducer workgroups of step t+1 sum fixed slices of them into
// level-2 sums (lvl_w); workgroup 0 of step t+2 sums those into the FP64
// accumulators.  Every sum runs in a fixed order.
struct StepLaunch {
  int precision, collision, path;
  const void* A;
  void* B;
  const uint32_t* links;
  const uint8_t* chunk;
  const double* inlet;
  void* part_w;             // slots of this step
  const void* part_r;       // slots of the previous step (reduced by this launch)
  double* lvl_w;            // level-2 sums written by this launch
  const double* lvl_r;      // level-2 sums of the step before the previous
  int reduce1;              // previous step's slots pending
  int reduce2;              // level-2 sums pending
  Acc* acc;
  double* hist;
  int64_t hist_cap;
  const MlpDev* mlp;
  const CbcDev* cbc;
  double* cbc_dt;           // [ny][4]: p_t, u_t, v_t of the last step at the outlet
  double* cbc_dt_w;         // two-step launches: where the launch leaves them
  int outlet;               // OUTLET_NN or OUTLET_CBC when n_nn > 0
  int nx, ny, pitch, nchunk;
  int64_t plane;
  int rows;             // rows per bulk block
  int ntx, nty;         // bulk tiles
  int n_nn;             // outlet blocks, neural or characteristic (0: Zou & He)
  int nspecial;         // 1 + kReducers + n_nn rounded up to a multiple of 8
  int nblocks;          // whole grid: nspecial + ntx*nty
  int xcd_chunk;        // bulk tiles per chunk dealt to the XCDs in turn (0: one band each)
  int pair_nslots;      // two-step launches: waves (slots per step), outlet blocks first
  int pair_nx;          // two-step launches: columns the bulk strips write
  int pair_out;         // two-step launches: outlet blocks (0: Zou & He in the strips)
  int pair_chunk;       // two-step launches: strip workgroups per chunk dealt to an XCD (0: eighths)
  int pair_rows;        // two-step launches: output rows per strip
  int pair_hold;        // two-step launches: step-(t+2) stores held one row (pair_hold)
  int tri_nslots;       // three-step launches: waves (slots per step), outlet blocks first
  int tri_nx;           // three-step launches: columns the strips write
  int tri_out;          // three-step launches: neural outlet blocks (0: Zou & He in the strips)
  int tri_chunk;        // three-step launches: strip workgroups per chunk dealt to an XCD
  int tri_rows;         // three-step launches: output rows per strip
  int tri_hold;         // three-step launches: step-(t+3) stores held one row (pair_hold's rule)
  int nslots;           // partial slots written per step (waves of the
                        // neural and bulk workgroups)
  int xper, yper;
  double omega, s_e, s_eps, s_q, u_in, one_minus_rho_out, n_fluid;
};

hipError_t launch_step(const StepLaunch& L, hipStream_t s);

// Record an error for lbm_last_error() (thread-local) and return `code`.
lbm_status set_error(lbm_status code, const char* fmt, ...);

// Per-node link words and per-(row, chunk) flags of a geometry mask (ny*nx,
// 0 fluid, 1 body, 2 inert solid) for a lattice of row pitch `pitch`;
// returns the number of fluid nodes.  links and chunk must be zeroed.
int64_t build_links(const uint8_t* mask, int nx, int ny, int pitch, int nchunk, bool xper,
                    bool yper, uint32_t* links, uint8_t* chunk);
hipError_t launch_finalize(const StepLaunch& L, hipStream_t s);
// Two steps per launch (Zou & He outflow only) and the flush after the last pair.
int pair_waves(int nx, int ny, int rows);
// Output rows per strip of the two-step kernel for an nx x ny lattice whose
// rows are pitch_bytes apart.
int pair_rows(int nx, int ny, int pitch_bytes);
// Whether the two-step strips hold their stores back by one row, for a
// lattice whose population buffer holds buffer_bytes.
int pair_hold(int precision, int64_t buffer_bytes);
// Two steps per launch with the neural outlet: outlet blocks for ny rows, and
// the columns at the outlet they take (the strips take the rest).
int pair_outlet_blocks(int ny);
// Strip workgroups per chunk dealt to the XCDs in turn (0: one eighth each).
int pair_chunk(int pair_nx);
int pair_outlet_cols();
hipError_t launch_pair(const StepLaunch& L, hipStream_t s);
hipError_t launch_finalize_pair(const StepLaunch& L, hipStream_t s);
// Three steps per launch (Zou & He outflow, FP32 and FP16 offsets).
int tri_waves(int nx, int ny, int rows);
// Output rows per strip of the three-step kernel; the strips and the
// outlet blocks of one launch share the four waves per SIMD of the rule.
int tri_rows(int nx, int ny, int pitch_bytes, int outlet_blocks);
int tri_chunk(int tri_nx);
// Outlet blocks of a three-step launch for ny rows (neural, or characteristic).
int tri_outlet_blocks(int ny, bool cbc);
bool tri_supported(int precision);
hipError_t launch_triple(const StepLaunch& L, hipStream_t s);
hipError_t launch_finalize_triple(const StepLaunch& L, hipStream_t s);

struct InitLaunch {
  int precision;
  void* A;
  void* B;
  const uint32_t* links;
  int nx, ny, pitch;
  int64_t plane;
  int y0, rows;              // row range
  const double* fields;      // staged rho, ux, uy [3][rows][nx], or null
  double u_in, noise_amp;
  uint64_t seed;
};
hipError_t launch_init(const InitLaunch& L, hipStream_t s);

// Copy rows [y0, y0+rows) of A to/from a dense FP64 staging array
// [9][rows][nx] of absolute populations.
hipError_t launch_read(int precision, const void* A, double* out, int nx, int pitch,
                       int64_t plane, int y0, int rows, hipStream_t s);
hipError_t launch_write(int precision, void* A, void* B, const double* in, int nx,
                        int pitch, int64_t plane, int y0, int rows, hipStream_t s);
// Moments (rho, ux, uy; Eq. 4) of rows [y0, y0+rows) of A into a dense FP64
// staging array [3][rows][nx].
hipError_t launch_macro(int precision, const void* A, double* out, int nx, int pitch,
                        int64_t plane, int y0, int rows, hipStream_t s);

// Standalone MLP evaluation on n feature rows (same device code as the fused
// outflow).
hipError_t launch_mlp_forward(const MlpDev* mlp, const float* x, float* s, int64_t n,
                              hipStream_t st);

}  // namespace lbm
