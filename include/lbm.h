/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice Boltzmann library.
 *
 * The library advances one two-dimensional D2Q9 lattice (or a batch of them)
 * by the time step of Bedrunka et al., "Reduction of Outflow Boundary
 * Influence on Aerodynamic Performance using Neural Networks":
 *
 *   stream + collide          Sec. 2.1, Eqs. 1-4 (BGK), MRT named in Sec. 3.2
 *   Zou & He columns          Sec. 2.2, Eqs. 5-11 (velocity inlet at x = 0,
 *                             pressure outlet at x = nx-1)
 *   bounce-back on solids     Sec. 2.3, Eq. 12, taken in its half-way form
 *   momentum-exchange force   Sec. 2.3, Eqs. 14-15
 *   neural outflow            Sec. 3.1, Eq. 16 (unknowns 3, 6, 7 at x = nx-1)
 *   MLP training              Sec. 3.1, Eq. 17
 *   characteristic outflow    Sec. 4, Eqs. 18-29 (fixed or network-tuned
 *                             sigma, kappa_2; periodic laterals)
 *
 * Conventions shared by every entry point
 *   - D2Q9 numbering q: 0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1)
 *     6 (-1,1) 7 (-1,-1) 8 (1,-1); weights 4/9, 1/9 x4, 1/36 x4.
 *   - x is streamwise (columns), y is transverse (rows); node centres at
 *     integers.  Host arrays are row-major: element (q, y, x) of a
 *     population array sits at q*ny*nx + y*nx + x; a scalar field (y, x) at
 *     y*nx + x.
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3, tau = 3 nu + 1/2.
 *   - Every call is asynchronous on the stream given in lbm_params unless
 *     its comment says it synchronises.  Host arrays passed in are copied
 *     before the call returns; host arrays passed out are filled before it
 *     returns.
 *   - Device memory: the caller allocates one workspace of
 *     lbm_workspace_bytes() bytes (256-byte aligned) and keeps it, and the
 *     stream, alive until lbm_destroy().  The library allocates no device
 *     memory of its own.
 *   - Errors: every call returns an lbm_status; a negative value is an
 *     error and lbm_last_error() then describes it (thread-local string,
 *     valid until the next call on that thread).  Argument errors are
 *     reported at once.  Faults and non-finite values inside kernels are
 *     reported by the next call that synchronises (lbm_forces,
 *     lbm_force_history, lbm_read_populations, lbm_sync).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;
typedef int32_t lbm_status;

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument or geometry                         */
  LBM_ENOSPACE = -2,   /* workspace smaller than lbm_workspace_bytes()     */
  LBM_EHIP = -3,       /* a HIP runtime call or kernel failed              */
  LBM_ESTATE = -4,     /* call out of order (e.g. step before geometry)    */
  LBM_EUNSTABLE = -5   /* a non-finite population or force was produced    */
};

enum { LBM_FP64 = 0, LBM_FP32_OFFSET = 1, LBM_FP16_OFFSET = 2 };
enum { LBM_BGK = 0, LBM_MRT = 1 };
enum { LBM_LATERAL_WALLS = 0, LBM_LATERAL_PERIODIC = 1 };
enum { LBM_X_INOUT = 0, LBM_X_PERIODIC = 1 };
enum { LBM_OUT_ZOUHE = 0, LBM_OUT_NN = 1, LBM_OUT_CBC = 2 };
/* Kernel schedule of lbm_step (the populations agree bit for bit, see
 * lbm_step). */
enum { LBM_LAUNCH_AUTO = 0, LBM_LAUNCH_SINGLE = 1, LBM_LAUNCH_PAIRS_PLAIN = 2,
       LBM_LAUNCH_PAIRS_HELD = 3, LBM_LAUNCH_TRIPLES = 4, LBM_LAUNCH_PAIRS = 5,
       LBM_LAUNCH_TRIPLES_PLAIN = 6, LBM_LAUNCH_TRIPLES_HELD = 7 };
/* Bulk tile of the one-step kernel: chosen by lattice size, or forced. */
enum { LBM_PATH_AUTO = 0, LBM_PATH_SCALAR = 1, LBM_PATH_VECTOR = 2 };

/*
 * Lattice description.
 *   nx, ny       lattice size, each >= 8 (nx >= 8 leaves room for the
 *                three-column stencil of the neural outflow).
 *   precision    storage of the populations: LBM_FP64 stores f_i - w_i in
 *                double and computes in double; LBM_FP32_OFFSET stores
 *                f_i - w_i in float and computes in float; LBM_FP16_OFFSET
 *                stores f_i - w_i in IEEE half and computes in float.
 *   collision    LBM_BGK (Eq. 2) or LBM_MRT (orthogonal moment basis rho, e,
 *                eps, jx, qx, jy, qy, pxx, pxy; equilibrium moments of Eq. 3;
 *                shear rate 1/tau).
 *   lateral      rows y = -1 and y = ny: half-way bounce-back walls, or
 *                periodic (Fig. 2).
 *   xbc          LBM_X_INOUT: Zou & He velocity inlet at x = 0 and outflow at
 *                x = nx-1 (Zou & He pressure or neural); LBM_X_PERIODIC:
 *                periodic in x (no inlet, no outlet).
 *   launch       LBM_LAUNCH_AUTO (0, the default): three time steps per
 *                kernel launch at FP32 and FP16 offsets (any outflow), two
 *                per launch at FP64, the rest of a count in two-step and
 *                single launches.  LBM_LAUNCH_TRIPLES: the same, rejected
 *                with LBM_FP64.  LBM_LAUNCH_PAIRS: two steps
 *                per launch only.
 *                LBM_LAUNCH_SINGLE: one launch per time step.  Two- and
 *                three-step launches walk their strips in one of two
 *                orders, chosen by lattice size (the stores of a row held
 *                back by one row above 200 MB per population buffer, FP32
 *                and FP64 only); LBM_LAUNCH_PAIRS_PLAIN / _HELD and
 *                LBM_LAUNCH_TRIPLES_PLAIN / _HELD take two- or three-step
 *                launches with one of them (HELD: not with
 *                LBM_FP16_OFFSET; TRIPLES: not with LBM_FP64).  Every
 *                schedule gives the same populations bit for bit.
 *   bulk_path    tile of the one-step kernel: LBM_PATH_AUTO (0: one node per
 *                thread below 12M nodes, four per lane above), or forced
 *                LBM_PATH_SCALAR / LBM_PATH_VECTOR.  Same results.
 *   tau          relaxation time, > 0.5.
 *   s_e, s_eps   MRT rates of the energy moments (ignored by BGK).
 *   s_q          MRT rate of the energy-flux moments; <= 0 selects
 *                1/(1/2 + (3/16)/(tau - 1/2)).
 *   u_in         inlet velocity (x component; the y component is 0).
 *   rho_out      outlet density of the Zou & He pressure condition.
 *   noise_amp    amplitude a of the initial velocity noise (see
 *                lbm_set_geometry).
 *   seed         SplitMix64 seed of that noise.
 *   history_cap  number of steps whose force is kept (0 keeps none).
 *   stream       hipStream_t, borrowed.
 */
typedef struct {
  int32_t nx, ny;
  int32_t precision, collision, lateral, xbc;
  int32_t launch, bulk_path;
  double tau, s_e, s_eps, s_q;
  double u_in, rho_out;
  double noise_amp;
  uint64_t seed;
  int64_t history_cap;
  void* stream;
} lbm_params;

/* Read-out of the force accumulators (lbm_forces).  Forces are in lattice
 * units (Eq. 15 with dx = dt = 1), summed over every link from a fluid node
 * into a body node (mask value 1). */
typedef struct {
  double fx, fy;          /* F(t) of the last step taken                    */
  double fx_sum, fy_sum;  /* sum of F over every step since the geometry    */
  double mass;            /* sum of rho over fluid nodes after the last step */
  int64_t step;           /* steps taken since lbm_set_geometry              */
  int64_t n_fallback;     /* neural-outflow nodes that fell back to Zou & He,
                             summed over steps                              */
  int32_t nonfinite;      /* 1 once a non-finite force or mass was seen     */
  int32_t reserved;
} lbm_force_out;

/* Weights of the outflow MLP n_in -> n_h1 -> n_h2 -> 3 (tanh, tanh, linear;
 * Sec. 3.1, Eq. 16), host arrays, FP32, row-major [out][in]:
 * w1 [n_h1][n_in], w2 [n_h2][n_h1], w3 [3][n_h2].  1 <= n_in <= 27,
 * 1 <= n_h1, n_h2 <= 64: a smaller network runs as the 27-64-64-3 one with
 * zero weights in the missing places (exactly the same result).  The paper's
 * own network is 9-20-20-3: the nine populations at x = L-1.
 * Inputs are the population offsets f_i - w_i at x = L-1, L-2, L-3 of the
 * outlet row (feature k = 9 j + q for column L-1-j; a network with n_in
 * inputs takes features 0 .. n_in-1), standardised as
 * z = (x - mu_in) * (1/sd_in) in FP32 and rounded to BF16.  Outputs are
 * s = o * sd_out + mu_out, the corrections of populations 3, 6, 7.
 * A node falls back to Zou & He unless every reconstructed population is
 * positive and |rho_g - rho(L-1)| < mass_bound. */
typedef struct {
  int32_t n_in, n_h1, n_h2, n_out;   /* n_in <= 27, n_h1, n_h2 <= 64, n_out = 3 */
  const float *w1, *b1, *w2, *b2, *w3, *b3;
  const float *mu_in, *sd_in, *mu_out, *sd_out;   /* [n_in], [n_in], [3], [3] */
  double mass_bound;
} lbm_mlp;

/* Workspace size in bytes for a lattice of these parameters. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a context on the caller's workspace.  Checks the parameters
 * (EINVAL) and the workspace size (ENOSPACE).  The lattice holds no state
 * until lbm_set_geometry. */
lbm_status lbm_create(const lbm_params* p, void* dev_workspace, size_t bytes,
                      lbm_ctx** out);

/* Wait for the work queued on the context's stream, then release the
 * context (not the workspace, which the caller owns and may free once this
 * returns).  NULL is a no-op. */
lbm_status lbm_destroy(lbm_ctx* c);

/* Upload the geometry and initialise the state.  host_mask is ny*nx bytes,
 * row-major: 0 fluid, 1 body (force-summed), 2 inert solid.  With
 * LBM_X_INOUT, columns 0 and nx-1 must be all fluid (EINVAL otherwise).
 * The state becomes f_i = f_i^eq(rho = 1, u) (Eq. 3), with
 * u = (u_in + a (2U - 1), a (2V - 1)) on fluid nodes and u = 0 on solid
 * nodes, where U and V are the SplitMix64 outputs k = 2 (y nx + x) + 1 and
 * k + 1 of the stream seeded with p->seed, mapped to [0, 1) by
 * (out >> 11) * 2^-53.  Resets the step count and force accumulators. */
lbm_status lbm_set_geometry(lbm_ctx* c, const uint8_t* host_mask);

/* Replace the state by f^eq(rho, u) from host fields rho, ux, uy (each ny*nx
 * doubles; solid nodes take f^eq(1, 0)).  Resets counters like
 * lbm_set_geometry. */
lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* ux,
                           const double* uy);

/* Per-row inlet velocity u_in(y) (ny doubles) instead of the uniform u_in;
 * NULL restores the uniform value. */
lbm_status lbm_set_inlet_profile(lbm_ctx* c, const double* host_ux);

/* Advance nsteps time steps (asynchronous).  One step: pull streaming of
 * the post-collision populations with half-way bounce-back on walls and
 * solids, the inlet and outlet columns, collision, and the force and mass
 * of the step (Sec. 2, Eqs. 1-4, 5-11, 12, 14-15).  Unless params.launch =
 * LBM_LAUNCH_SINGLE, two or three steps run in each launch (params.launch)
 * with the same node arithmetic and every intermediate state rounded to the
 * storage precision as a store would round it, so the populations equal
 * those of one launch per step bit for bit and the force and mass sums
 * agree to their rounding; a count that does not divide ends with a
 * two-step or single launch.  ESTATE before lbm_set_geometry. */
lbm_status lbm_step(lbm_ctx* c, int64_t nsteps);

/* Synchronise the stream and read the accumulators.  Returns EUNSTABLE
 * (with *out filled) once a non-finite force or mass has been seen. */
lbm_status lbm_forces(lbm_ctx* c, lbm_force_out* out);

/* Synchronise and copy the per-step force history F(t), t = 0 .. n-1
 * (n = min(steps, history_cap, cap)), into fx, fy (host, cap doubles). */
lbm_status lbm_force_history(lbm_ctx* c, double* fx, double* fy, int64_t cap,
                             int64_t* n);

/* Select the outflow at x = nx-1: LBM_OUT_ZOUHE (w ignored, may be NULL) or
 * LBM_OUT_NN with the weights *w, which are copied (rounded to BF16).  The
 * characteristic outflow is selected by lbm_set_outflow_cbc. */
lbm_status lbm_set_outflow_model(lbm_ctx* c, int32_t kind, const lbm_mlp* w);

/* Tuning network of the characteristic outflow (Sec. 4.2): nine features per
 * outlet node, (p_x, u_x, v_x, p_y, u_y, v_y, p_t, u_t, v_t), the time
 * derivatives being those the outflow computed at the previous step (zero
 * before the first), standardised z = (x - mu_in) / sd_in; two hidden layers
 * of 20 with LeakyReLU (negative slope leaky_slope); two outputs s_0, s_1;
 * sigma = sigma_scale * sigmoid(s_0) + sigma_shift and
 * kappa_2 = kappa_scale * sigmoid(s_1) + kappa_shift.  Host FP32 arrays,
 * row-major [out][in]: w1 [20][9], w2 [20][20], w3 [2][20]; evaluated in the
 * arithmetic precision of the lattice. */
typedef struct {
  const float *w1, *b1, *w2, *b2, *w3, *b3;
  const float *mu_in, *sd_in;            /* [9] each, sd_in > 0 */
  double leaky_slope;
  double sigma_scale, sigma_shift, kappa_scale, kappa_shift;
} lbm_cbc_net;

/* Characteristic outflow (Sec. 4, Eqs. 18-29).  At every step the outlet
 * node takes the density and velocity of a forward Euler step of the
 * isothermal LODI equations (Eqs. 18-20) from the state of columns nx-3 ..
 * nx-1 (one-sided x-derivatives of second order, central y-derivatives),
 * with the incoming amplitude
 * L_1 = kappa_1 (p - p_inf) - kappa_2 T_1 + T_1, kappa_1 = sigma (1 - M^2)
 * c_s / L (Eqs. 27-28; p = rho / 3, p_inf = rho_inf / 3); the unknown
 * populations then follow from Eqs. 8-10 for that state, after f_0 is
 * corrected so that the node carries the density exactly (Eq. 29).  With
 * net == NULL sigma and kappa_2 are the fixed values below, else the network
 * sets them per node and step (the network is copied).  Needs LBM_X_INOUT,
 * LBM_LATERAL_PERIODIC (the section defines no treatment of the corners
 * where the outlet meets a wall; EINVAL otherwise) and fluid in the last
 * three columns.  Selecting it clears the stored time derivatives. */
typedef struct {
  double sigma, kappa2;     /* fixed tuning parameters (ignored with net)     */
  double mach;              /* M in kappa_1, 0 <= M < 1                        */
  double length;            /* L in kappa_1 (> 0), e.g. the lattice length     */
  double rho_inf;           /* far-field density (> 0)                        */
  const lbm_cbc_net* net;   /* NULL: fixed sigma, kappa_2                     */
} lbm_cbc;

lbm_status lbm_set_outflow_cbc(lbm_ctx* c, const lbm_cbc* p);

/* Synchronise and write the moments of the stored state (Eq. 4), FP64, to
 * host arrays of ny*nx doubles, row-major: rho = sum_i f_i, ux = sum_i c_ix
 * f_i / rho, uy = sum_i c_iy f_i / rho, summed in FP64 from the stored values
 * (collision conserves them, so they are also the moments before the
 * collision of the last step).  Solid nodes give rho = 1, u = 0 (their
 * stored equilibrium).  ESTATE before lbm_set_geometry. */
lbm_status lbm_read_macroscopic(lbm_ctx* c, double* rho, double* ux, double* uy);

/* Synchronise and copy the stored state -- the post-collision populations
 * f*(t) of the last step, as absolute values f_i (not offsets) -- into host
 * (9*ny*nx doubles).  Solid nodes hold their initial equilibrium. */
lbm_status lbm_read_populations(lbm_ctx* c, double* host);

/* Replace the stored post-collision state by host (9*ny*nx doubles,
 * absolute values), rounded to the storage precision.  The step count and
 * accumulators are kept. */
lbm_status lbm_write_populations(lbm_ctx* c, const double* host);

/* Synchronise the stream; reports kernel faults (EHIP). */
lbm_status lbm_sync(lbm_ctx* c);

/* Evaluate the outflow MLP of the context on n feature rows (device
 * pointers): x [n][27] FP32 population offsets (a network with fewer inputs
 * reads the first n_in of each row, the rest must be finite), s [n][3] FP32 outputs
 * (corrections of populations 3, 6, 7).  Same kernels and roundings as the
 * fused outflow.  ESTATE unless an LBM_OUT_NN model is set. */
lbm_status lbm_mlp_forward(lbm_ctx* c, const float* dev_x, float* dev_s,
                           int64_t n);

/* Description of the last error on this thread. */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
