/*
 * lbpf — phase-field lattice Boltzmann two-phase solver for AMD Instinct MI355X (gfx950).
 *
 * Method: Yuan, Chai, Wang & Shi, "A generalized lattice Boltzmann model for fluid flow system
 * and its application in two-phase flows" (arXiv:1902.08933), Sec. 3: the D2Q9 hydrodynamic
 * distribution of eq. (24) with equilibrium eq. (33), force distribution eq. (34), velocity
 * eq. (27a) and modified pressure eq. (28) (or eq. (29)), coupled to the Cahn-Hilliard
 * distribution of eq. (10) with equilibrium eq. (11), source eq. (14) and order parameter
 * eq. (18); the closure of Sec. 3.1 (eq. 3aa density, eq. 8 chemical potential) and the
 * isotropic stencils of eqs. (30a)-(30b). Quasi-incompressible (S1 = -gamma div(M grad mu),
 * Sec. 3.2.1) and incompressible (S1 = 0) variants.
 *
 * Conventions shared by every call:
 *  - Grids are row-major [ny][nx] with x fastest; nodes sit at integer (i, j), lattice units
 *    dx = dt = 1, c_s^2 = 1/3. phi = 1 is phase A, phi = 0 is phase B (Sec. 3.1).
 *  - Device pointers are HIP device addresses. The library never allocates device memory:
 *    the caller passes one device workspace of lbpf_workspace_size() bytes and keeps it alive
 *    until lbpf_destroy(). The library owns only its host-side handle.
 *  - All work is enqueued on the caller's HIP stream (hipStream_t passed as void*; NULL means
 *    the legacy default stream). Calls return after enqueueing unless stated otherwise.
 *  - Every call returns an lbpf_status; LBPF_OK is 0. No C++ exception crosses the ABI.
 *    On failure lbpf_last_error() returns a message for that handle.
 *  - One handle must not be used from two host threads at once; distinct handles are
 *    independent.
 */
#ifndef LBPF_H
#define LBPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBPF_OK = 0,
    LBPF_E_INVALID = -1,  /* bad argument or parameter (message says which) */
    LBPF_E_HIP = -2,      /* a HIP runtime call failed (message holds the HIP error string) */
    LBPF_E_NOMEM = -3,    /* workspace or buffer too small, or host allocation failed */
    LBPF_E_UNSTABLE = -4, /* diagnostics found a non-finite value in the state */
    LBPF_E_STATE = -5     /* call out of order (e.g. step before init) */
} lbpf_status;

/* Sec. 4 introduction: incompressible (S1 = 0) or quasi-incompressible
 * (S1 = -gamma div(M_phi grad mu), gamma = (rho_A - rho_B) / rho_B, Sec. 3.2.1). */
typedef enum { LBPF_QIM = 0, LBPF_IM = 1 } lbpf_variant;

/* Pressure: eq. (28) with G_0 taken from eq. (34) at i = 0 (default); eq. (28) with the
 * simplified G_0 printed after eq. (34); or eq. (29), which drops the G_0 term. */
typedef enum { LBPF_P_EQ28 = 0, LBPF_P_EQ28_PAPER_G0 = 1, LBPF_P_EQ29 = 2 } lbpf_pscheme;

/* Surface tension: F_s = mu grad(phi) (Sec. 3.1, default) or F_s = -phi grad(mu) (Sec. 4.2). */
typedef enum { LBPF_FS_MU_GRADPHI = 0, LBPF_FS_NEG_PHI_GRADMU = 1 } lbpf_fsurf;

/* Viscosity across the interface: inverse-linear in 1/nu (after eq. 17), or a step in the
 * dynamic viscosity mu = rho nu at phi = 1/2 (Sec. 4.3). */
typedef enum { LBPF_VISC_INVLIN = 0, LBPF_VISC_STEP = 1 } lbpf_visc;

/* Boundaries: fully periodic, or periodic in x with halfway bounce-back walls half a cell
 * below row 0 and above row ny-1 (Sec. 4.3). Stencils mirror the first fluid row at a wall. */
typedef enum { LBPF_BC_PERIODIC = 0, LBPF_BC_WALLS_Y = 1 } lbpf_bc;

/* Macroscopic fields of the current state (lbpf_read). */
typedef enum {
    LBPF_FIELD_PHI = 0, /* eq. (18) */
    LBPF_FIELD_RHO = 1, /* eq. (3aa) */
    LBPF_FIELD_UX = 2,  /* eq. (27a) */
    LBPF_FIELD_UY = 3,
    LBPF_FIELD_P = 4,   /* eq. (28) or (29), evaluated on the current state */
    LBPF_FIELD_MU = 5   /* eq. (8) */
} lbpf_field;

/* Physical parameters of one simulation (lattice units). */
typedef struct lbpf_params {
    int32_t nx, ny;          /* grid size: 3 <= nx, ny < 2^24 and ny * pitch(nx) + pad < 2^30,
                              * pitch(nx) = nx rounded up to a multiple of 64 */
    int32_t variant;         /* lbpf_variant */
    int32_t pscheme;         /* lbpf_pscheme */
    int32_t fsurf;           /* lbpf_fsurf */
    int32_t visc;            /* lbpf_visc */
    int32_t bc;              /* lbpf_bc */
    int32_t clamp_props;     /* nonzero: phi clamped to [0,1] where rho(phi), nu(phi) are evaluated */
    double rho_A, rho_B;     /* densities of phase A (phi = 1) and B (phi = 0), > 0 */
    double nu_A, nu_B;       /* kinematic viscosities, > 0 (relaxation tau_g = 3 nu + 1/2) */
    double sigma, W;         /* surface tension >= 0 and interface width > 0 (eqs. 6-7) */
    double M_phi;            /* mobility (eq. 17) */
    double tau_h;            /* Cahn-Hilliard relaxation time, > 1/2 (eq. 10) */
    double force_x, force_y; /* constant body-force density */
    double gravity;          /* buoyancy F_y = -(rho - rho_A) * gravity (Sec. 4.4) */
} lbpf_params;

/* Conserved-quantity diagnostics, reduced in FP64 on the GPU in a fixed order. */
typedef struct lbpf_diag {
    double sum_phi;    /* sum over nodes of phi = sum_i h_i (globally conserved, Sec. 3.2.2) */
    double sum_rho;    /* sum over nodes of rho(phi) */
    double max_u;      /* max over nodes of |u| */
    int64_t nonfinite; /* number of non-finite values in the stored state */
    int64_t step;      /* time steps taken since lbpf_init */
} lbpf_diag;

typedef struct lbpf_ctx lbpf_ctx;

/* Bytes of device workspace a simulation with these parameters needs: two ping-pong copies of
 * the state (f_1..8, h_0 hi/lo and h_1..8, pressure and (phi u) histories; 21 planes each,
 * interleaved by grid row, or as separate planes for grids above about 7100^2 or when the
 * environment sets LBPF_STATE_LAYOUT=planar), an FP64 scratch and the reduction area. The layout
 * must not change between this call and lbpf_create. */
lbpf_status lbpf_workspace_size(const lbpf_params* params, size_t* bytes);

/* Validate params and bind a handle to a caller-owned device workspace and stream.
 * Rejects nx or ny < 3, tau_h <= 1/2, nu <= 0, rho <= 0, W <= 0, sigma < 0 with
 * LBPF_E_INVALID, and a workspace smaller than lbpf_workspace_size() with LBPF_E_NOMEM.
 * On failure *out is NULL and lbpf_create_error() describes the reason. */
lbpf_status lbpf_create(const lbpf_params* params, void* workspace, size_t workspace_bytes,
                        void* hip_stream, lbpf_ctx** out);

/* Initial state from device fields [ny][nx] FP32 (any of ux, uy, p may be NULL for zero):
 * h_i = h_i^eq(phi0, mu0, u0) (eq. 11) with mu0 from eq. (8), g_i = g_i^eq(p0, rho(phi0), u0)
 * (eq. 33); the (phi u) and pressure histories start at phi0 u0 and p0. Resets the step count. */
lbpf_status lbpf_init(lbpf_ctx* ctx, const float* phi, const float* ux, const float* uy,
                      const float* p);

/* Advance nsteps >= 0 time steps (eq. 24 and eq. 10 with streaming). Asynchronous. */
lbpf_status lbpf_step(lbpf_ctx* ctx, int64_t nsteps);

/* Write one lbpf_field of the current state to a device array [ny][nx] FP32. Asynchronous. */
lbpf_status lbpf_read(lbpf_ctx* ctx, int32_t field, float* dst);

/* FP64 diagnostics of the current state; synchronizes the stream. Returns LBPF_E_UNSTABLE
 * (with *out filled) when a stored value is not finite. */
lbpf_status lbpf_diagnostics(lbpf_ctx* ctx, lbpf_diag* out);

/* lbpf_diagnostics for callers that cannot allocate device memory (code under graph capture,
 * allocation-free serving loops): the same kernels and results, bitwise, but the reduction
 * partials live in a fixed device array of the library (263 KB per GPU, held until the process
 * ends) instead of the handle's workspace. Every call on one GPU shares that array and leaves its
 * contents behind; the partials are rewritten by each call, so nothing needs clearing, and calls
 * that overlap on one GPU (two streams, two threads) race. Allocates nothing; LBPF_E_NOMEM if the
 * partials would not fit the array (they always fit: at most 4096 blocks). Synchronizes the
 * stream. */
lbpf_status lbpf_diagnostics_noalloc(lbpf_ctx* ctx, lbpf_diag* out);

/* FP64 statistics of one lbpf_field of the current state over all nodes: out3[0] the mean,
 * out3[1] the standard deviation about it, out3[2] the largest magnitude. Reduced on the GPU in
 * a fixed order; synchronizes the stream. (Used to normalize the fields handed to the learned
 * surrogate; equally a diagnostic of the state.) */
lbpf_status lbpf_field_stats(lbpf_ctx* ctx, int32_t field, double* out3);

/* lbpf_field_stats of n (1 to 6) fields at once, with one synchronization: out (3 n doubles,
 * host) receives for field[k] its mean, standard deviation and largest magnitude at out[3 k],
 * bit for bit what lbpf_field_stats returns for it. LBPF_E_INVALID for n out of range, an unknown
 * field or NULL arrays. (The hybrid surrogate reads the statistics of five fields per cycle.) */
lbpf_status lbpf_field_stats_many(lbpf_ctx* ctx, int32_t n, const int32_t* field, double* out);

/* Laplace-law pressure jump of Sec. 4.2 in FP64: P = p0 - kappa phi lap(phi)
 * + kappa |grad phi|^2 / 2 + p with p0 = phi psi'(phi) - psi(phi), averaged over nodes with
 * periodic distance r <= R/2 from (xc, yc) minus the average over r >= R + 3W.
 * Synchronizes the stream. */
lbpf_status lbpf_laplace_dp(lbpf_ctx* ctx, double xc, double yc, double R, double* dP);

/* Checkpoint: bytes of the current state (populations, histories, step count). */
lbpf_status lbpf_state_size(const lbpf_ctx* ctx, size_t* bytes);
/* Copy the current state into / out of a caller device buffer of lbpf_state_size() bytes
 * (a 64-byte header, then the state copy as stored). Asynchronous; a save followed by a load on
 * another handle with equal params and layout resumes bit-identically; a checkpoint of another
 * grid or layout is refused with LBPF_E_INVALID. */
lbpf_status lbpf_save_state(lbpf_ctx* ctx, void* dst_device);
lbpf_status lbpf_load_state(lbpf_ctx* ctx, const void* src_device);

/* Change the stream used by later calls. */
lbpf_status lbpf_set_stream(lbpf_ctx* ctx, void* hip_stream);

/* Work shape of the fused step: index into the list of strip shapes. A workgroup of `threads`
 * threads owns a strip `tx` nodes wide and `rows` rows tall and marches up it. Results are
 * bit-identical for every shape. A new simulation starts with shape 12 (64 x 32, 512 threads),
 * a new batch with shape 1 (64 x 16, 256 threads); the autotuners below pick per workload. */
lbpf_status lbpf_set_tile(lbpf_ctx* ctx, int32_t tile_index);
/* Autotuner: times every strip shape over trial_steps steps (after one warm-up launch each)
 * on this simulation's own grid and parameters, writes the mean milliseconds per step of shape i
 * to ms_out[i] (may be NULL; else lbpf_tile_count() floats), selects the fastest shape and
 * returns its index in *best_out. The state is saved to scratch_state (a device buffer of
 * lbpf_state_size() bytes) first and restored afterwards, step count included, so the tuned
 * simulation continues bit-identically. Synchronizes the stream. */
lbpf_status lbpf_autotune(lbpf_ctx* ctx, int32_t trial_steps, void* scratch_state, float* ms_out,
                          int32_t* best_out);
/* Strip shape in use (-1 for a NULL handle). */
int32_t lbpf_get_tile(const lbpf_ctx* ctx);
/* Number of strip shapes, and the (tx, rows, threads) triple of one of them. */
int32_t lbpf_tile_count(void);
lbpf_status lbpf_tile_shape(int32_t tile_index, int32_t* tx, int32_t* rows, int32_t* threads);

int64_t lbpf_step_count(const lbpf_ctx* ctx);

/* HBM bandwidth probe (the reference point of the roofline): mode 0 copies `bytes` from src to
 * dst, mode 1 reads src (dst must hold one float per workgroup; it is written only when a
 * partial sum equals an improbable sentinel), mode 2 writes zeros to dst. 16-byte accesses, grid-stride over `blocks` workgroups of
 * 256 threads (blocks <= 0: 4096). bytes must be a multiple of 16; buffers are caller-owned
 * device memory. Asynchronous on hip_stream; errors via lbpf_create_error(). */
lbpf_status lbpf_bw_probe(int32_t mode, const void* src, void* dst, size_t bytes, int32_t blocks,
                          void* hip_stream);

/* Release the handle (does not free the caller's workspace). NULL is accepted. */
lbpf_status lbpf_destroy(lbpf_ctx* ctx);

const char* lbpf_status_string(lbpf_status status);
/* Message of the last failed call on this handle; valid until the next call on it. */
const char* lbpf_last_error(const lbpf_ctx* ctx);
/* Message of the last failed lbpf_create / lbpf_workspace_size on this thread. */
const char* lbpf_create_error(void);

/* ------------------------------------------------------------------------------------------
 * Batch: many independent simulations (own grid size and parameters each) advanced together by
 * one persistent kernel per time step, replayed from HIP graphs of 8 steps. Each instance
 * evolves bit-identically to a single simulation with the same parameters and initial fields.
 * Instances are addressed by index 0..n-1; lbpf_batch_instance() returns the per-instance
 * handle for lbpf_read, lbpf_diagnostics, lbpf_laplace_dp and checkpointing (not for lbpf_step
 * or lbpf_init: use the batch calls). The batch owns those handles.
 * ------------------------------------------------------------------------------------------ */
typedef struct lbpf_batch lbpf_batch;

/* Device workspace bytes for n instances with parameters params[0..n-1]: the instance table,
 * the work list, 8 x 8 work counters of the batched kernel, then each instance's workspace. */
lbpf_status lbpf_batch_workspace_size(int32_t n, const lbpf_params* params, size_t* bytes);
/* Bind a batch to a caller-owned workspace (256-byte aligned) and stream; builds the work
 * list of (instance, strip chunk) items and the step graphs. Errors as lbpf_create. */
lbpf_status lbpf_batch_create(int32_t n, const lbpf_params* params, void* workspace,
                              size_t workspace_bytes, void* hip_stream, lbpf_batch** out);
/* Initial state of instance idx, as lbpf_init; also clears a frozen flag. */
lbpf_status lbpf_batch_init(lbpf_batch* b, int32_t idx, const float* phi, const float* ux,
                            const float* uy, const float* p);
/* Advance every instance nsteps steps. Launches use the 8 work-counter slots of the workspace
 * in cyclic order: single launches until slot 0 comes round, graph replays of 8 steps (slots
 * 0..7), then single launches. Every instance must be initialized. Asynchronous; steps of one
 * batch must not be issued on two streams at once (they share the counters). */
lbpf_status lbpf_batch_step(lbpf_batch* b, int64_t nsteps);
/* Reference path: the same steps with one single-simulation launch per instance per step (a
 * frozen instance is skipped), for comparison with lbpf_batch_step. */
lbpf_status lbpf_batch_step_each(lbpf_batch* b, int64_t nsteps);
/* Per-instance FP64 diagnostics (flags[k] = 1 for a frozen instance). An instance whose state
 * holds a non-finite value is frozen: it leaves the work list (rebuilt here), later steps leave
 * its state and step count as they are while the others go on, and lbpf_batch_init brings it
 * back. flags (n int32) and diags (n lbpf_diag) may be NULL. Synchronizes the stream. */
lbpf_status lbpf_batch_status(lbpf_batch* b, int32_t* flags, lbpf_diag* diags);
lbpf_ctx* lbpf_batch_instance(lbpf_batch* b, int32_t idx);
int32_t lbpf_batch_count(const lbpf_batch* b);
/* Strip shape of the batched kernel (rebuilds the work list and graphs); results are
 * bit-identical for every shape. */
lbpf_status lbpf_batch_set_tile(lbpf_batch* b, int32_t tile_index);
int32_t lbpf_batch_get_tile(const lbpf_batch* b);
/* Bytes of a buffer holding every instance state (for lbpf_batch_autotune). */
lbpf_status lbpf_batch_state_size(const lbpf_batch* b, size_t* bytes);
/* Autotuner for the batch: times every strip shape over trial_steps steps, keeps the fastest
 * (ms_out as in lbpf_autotune), and restores every instance state from scratch_state
 * (lbpf_batch_state_size() bytes of device memory). Synchronizes the stream. */
lbpf_status lbpf_batch_autotune(lbpf_batch* b, int32_t trial_steps, void* scratch_state,
                                float* ms_out, int32_t* best_out);
int64_t lbpf_batch_step_count(const lbpf_batch* b);
lbpf_status lbpf_batch_destroy(lbpf_batch* b);
const char* lbpf_batch_last_error(const lbpf_batch* b);

/* ------------------------------------------------------------------------------------------
 * Learned surrogate: a 4-level convolutional U-Net (level widths base_ch << l, l = 0..3; 3x3
 * convolutions with circular padding, 2x2 average pooling, nearest upsampling, skip
 * concatenation, 1x1 head) mapping the fields (phi, u_x, u_y, p) of the solver at time t to
 * time t + K. It adds a predicted change to its input. BF16 weights and activations, FP32
 * accumulation on MFMA, FP32 master weights and Adam moments. Fields are FP32 NHWC
 * [n][h][w][in_ch] device arrays; h and w multiples of 8. Errors via lbpf_unet_last_error().
 * ------------------------------------------------------------------------------------------ */
typedef struct lbpf_unet lbpf_unet;
typedef struct lbpf_unet_cfg {
    int32_t in_ch;        /* field channels, 1..16 (4: phi, u_x, u_y, p) */
    int32_t base_ch;      /* width of level 0 (16, 32, ... 128); 32 gives ~0.97 M parameters */
    int32_t max_batch;    /* largest n * h * w the workspace holds is max_batch*max_h*max_w */
    int32_t max_h, max_w; /* multiples of 8 */
    int32_t train;        /* nonzero: workspace includes gradients and Adam moments */
    int32_t wgrad_chunks; /* size of the weight-gradient partial buffers, in pixel chunks of the
                           * largest layer (0: 64); smaller layers use proportionally more chunks */
    int32_t pad;
    uint64_t seed;        /* He-normal initial weights; the head starts at zero */
} lbpf_unet_cfg;

lbpf_status lbpf_unet_workspace_size(const lbpf_unet_cfg* cfg, size_t* bytes);
lbpf_status lbpf_unet_create(const lbpf_unet_cfg* cfg, void* workspace, size_t workspace_bytes,
                             void* hip_stream, lbpf_unet** out);
int64_t lbpf_unet_param_count(const lbpf_unet* u);
/* Layer i (0..7: encoder 0..3, decoder 2, 1, 0, head): offsets of its weights
 * [cout][ks*ks][cin] and bias [cout] in the flat FP32 parameter vector. */
lbpf_status lbpf_unet_layer(const lbpf_unet* u, int32_t i, int64_t* woff, int64_t* boff,
                            int32_t* cout, int32_t* ks, int32_t* cin);
/* Copy the FP32 master parameters out of / into the network (device arrays of
 * lbpf_unet_param_count() floats); setting also resets the Adam moments. */
lbpf_status lbpf_unet_get_params(lbpf_unet* u, float* dst_device);
lbpf_status lbpf_unet_set_params(lbpf_unet* u, const float* src_device);
/* Per-channel weights of the squared-error loss (16 host floats; channels >= in_ch ignored). */
lbpf_status lbpf_unet_set_loss_weights(lbpf_unet* u, const float* host_weights);
/* Inference: out = in + net(in). Asynchronous. */
lbpf_status lbpf_unet_forward(lbpf_unet* u, const float* in, float* out, int32_t n, int32_t h,
                              int32_t w);
/* Loss (mean over pixels and in_ch channels of w_c (out - target)^2) and its gradient with
 * respect to the flat parameters (grad_device may be NULL). Synchronizes the stream. */
lbpf_status lbpf_unet_loss_grad(lbpf_unet* u, const float* in, const float* target, int32_t n,
                                int32_t h, int32_t w, double* loss_host, float* grad_device);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) on the loss above; *loss_host before the update. */
lbpf_status lbpf_unet_train_step(lbpf_unet* u, const float* in, const float* target, int32_t n,
                                 int32_t h, int32_t w, float lr, double* loss_host);
lbpf_status lbpf_unet_destroy(lbpf_unet* u);
const char* lbpf_unet_last_error(const lbpf_unet* u);
/* One 16 x 16 x k BF16 matrix product on MFMA, k = 16 or 32 (row-major A 16 x k and B k x 16
 * bf16, D 16 x 16 FP32, device arrays): the operand-layout check of the surrogate kernels. */
lbpf_status lbpf_mfma_probe(int32_t k, const void* A, const void* B, float* D, void* hip_stream);

/* One convolution of the surrogate network run by the kernel the network's layers use, chosen by
 * the same rules from the sizes: the check of the convolution kernels on caller tensors, layer by
 * layer. out[p, co] = bias[co] + sum_{tap, ci} in[p + off(tap), ci] wt[co][tap][ci] with circular
 * padding (off(tap) = (tap / 3 - 1, tap % 3 - 1) for ks = 3, (0, 0) for ks = 1), FP32
 * accumulation, then ReLU if asked. The input channels are [up(xl), x]: channels [0, cl) the
 * nearest 2x upsampling of xl, channels [cl, cin) from x; or, in first-layer mode (xin set,
 * ks = 3, cl = 0), the bf16 rounding of the FP32 fields of xin, cin being then the weights'
 * channel stride. Outputs (each optional, all NHWC device arrays): y the bf16 rounding (to
 * nearest even) of out; yp the bf16 rounding of the mean of each 2 x 2 block of y (h, w even);
 * yf out in FP32; pred = res + out[:, :rc], or with hw set (cout <= 32) res + hb + the 1 x 1
 * head hw [rc][cout] applied to y. Channel counts, cl and cin - cl multiples of 8 except in
 * first-layer mode. variant (3 int32, may be NULL) receives the kernel chosen: tiled (0),
 * first-layer (1), wave-row (2, ks = 3 with cin, cl and cout multiples of 32) or persistent
 * first-layer (3: 4 fields, cout 32, y and/or yp only, h and w multiples of 16), the output
 * channels per workgroup (16, 32, 64 or 128), and 1 if the tiled kernel prefetches the next
 * input chunk's weights into registers or the wave-row kernel's work items are 8 rows high
 * instead of 16. Asynchronous; LBPF_E_INVALID for shapes the kernels do
 * not take. Defined by the network description above; used by its tests. */
typedef struct lbpf_unet_conv_desc {
    int32_t ks, relu;  /* 1 or 3; nonzero: ReLU after the bias */
    int32_t n, h, w;   /* images and their size */
    int32_t cin, cl;   /* input channels; the first cl of them upsampled from xl */
    int32_t cout;      /* output channels */
    int32_t xin_c;     /* first-layer mode: fields of xin (1..4) */
    int32_t rc;        /* channels of res and pred (1..16) */
    const void* x;     /* bf16 [n][h][w][cin - cl] */
    const void* xl;    /* bf16 [n][h/2][w/2][cl] */
    const float* xin;  /* FP32 [n][h][w][xin_c] */
    const void* wt;    /* bf16 [cout][ks*ks][cin] */
    const float* bias; /* FP32 [cout] or NULL */
    void* y;           /* bf16 [n][h][w][cout] */
    void* yp;          /* bf16 [n][h/2][w/2][cout] */
    float* yf;         /* FP32 [n][h][w][cout] */
    const float* res;  /* FP32 [n][h][w][rc] */
    float* pred;       /* FP32 [n][h][w][rc] */
    const void* hw;    /* bf16 [rc][cout] */
    const float* hb;   /* FP32 [rc] or NULL */
} lbpf_unet_conv_desc;
lbpf_status lbpf_unet_conv_probe(const lbpf_unet_conv_desc* desc, int32_t* variant, void* hip_stream);
/* The weight and bias gradients of one such convolution (ks 1 or 3, no upsampled part) as the
 * network's backward pass computes them: dw[co][tap][ci] = sum_p dy[p, co] x[p + off(tap), ci]
 * and db[co] = sum_p dy[p, co] (FP32), with dy bf16 [n][h][w][cout] and x bf16 [n][h][w][cin],
 * from per-chunk partials summed in a fixed order. part and bpart are caller device scratch of
 * max_chunks * cout * ks*ks * cin and max_chunks * cout floats. cin, cout multiples of 8.
 * Asynchronous. */
lbpf_status lbpf_unet_wgrad_probe(int32_t ks, const void* dy, const void* x, int32_t n, int32_t h,
                                  int32_t w, int32_t cin, int32_t cout, int32_t max_chunks,
                                  float* part, float* bpart, float* dw, float* db, void* hip_stream);

/* Hand-over between the solver and the surrogate: the current fields of a simulation as
 * normalized NHWC [ny][nx][4] FP32, (field - shift[c]) / scale[c] for c = phi, u_x, u_y, p
 * (host arrays of 4; dst 16-byte aligned); and a new state from such fields at time level
 * `step` (equilibria as in lbpf_init; the histories start from the given fields). Async. */
lbpf_status lbpf_fields_to_nhwc(lbpf_ctx* ctx, float* dst, const float* shift, const float* scale);
lbpf_status lbpf_init_from_nhwc(lbpf_ctx* ctx, const float* src, const float* shift,
                                const float* scale, int64_t step);

/* ------------------------------------------------------------------------------------------
 * Generalized single-phase model with a mass source (Sec. 2): the evolution eq. (24), the
 * equilibrium eq. (25) and the force term eq. (27), with the velocity eq. (27a), in the two
 * reductions the paper spells out:
 *   LBPF_SP_NEARLY_INCOMPRESSIBLE  Remark 1: rho~ = rho = sum_i g_i + S/2 (eq. 27aa),
 *       p = rho c_s^2, g_i^eq = rho [w_i + s_i(u)] (eq. 29bb); force bracket
 *       uF + Fu - uu S + Q (div u) I, with div u of the previous step's velocity (eq. 30a).
 *   LBPF_SP_INCOMPRESSIBLE  Remark 3: rho~ = rho0, rho = 1, g^eq of eq. (25), p by eq. (28)
 *       (or eq. 29); force bracket uF + Fu + Q S I. With `full`, the terms of eq. (27) that
 *       Remark 3 neglects are kept: -grad p^{n-1} (eq. 30a) in F~, -uu S, and d_t p I with
 *       d_t p = p^n - p^{n-1}, for which eq. (28) is solved in closed form (G_0 is affine in it).
 * Q = (2/d) rho c_s^2 - xi / (tau_g - 1/2), tau_g = nu / c_s^2 + 1/2. S(x) and F(x) are fields
 * given at lbpf_sp_init and constant in time. Same conventions as the two-phase solver: the
 * caller owns the device workspace and the stream; calls are asynchronous unless stated.
 * ------------------------------------------------------------------------------------------ */
typedef enum { LBPF_SP_NEARLY_INCOMPRESSIBLE = 0, LBPF_SP_INCOMPRESSIBLE = 1 } lbpf_sp_model;
typedef enum { LBPF_SP_RHO = 0, LBPF_SP_UX = 1, LBPF_SP_UY = 2, LBPF_SP_P = 3 } lbpf_sp_field;

typedef struct lbpf_sp_params {
    int32_t nx, ny;   /* same limits as lbpf_params */
    int32_t model;    /* lbpf_sp_model */
    int32_t pscheme;  /* incompressible model: 0 eq. (28), 1 eq. (29) */
    int32_t full;     /* 1: force term as printed (see above); 0: the Remarks' reduced forms
                       * (nearly incompressible: -uu S dropped) */
    int32_t bc;       /* lbpf_bc */
    double nu;        /* kinematic viscosity (> 0) */
    double xi;        /* bulk viscosity (0: Stokes hypothesis) */
    double rho0;      /* incompressible model: the constant rho~ */
    double drag;      /* nearly incompressible model: lambda >= 0 makes the force
                       * F = F_ext - lambda rho u, a force that depends on u; eq. (27a) is then
                       * implicit and, being linear, solved in closed form */
    int32_t scheme;   /* nearly incompressible model: 0 eq. (24) on g = f~ - G/2 (eq. 23a);
                       * 1 Remark 4, the explicit discretization of D_i G_i on f~ itself
                       * (rho~ = sum f~, rho u = sum c f~; stores G of the previous step;
                       * G_i(x + c_i) across a wall is taken at x; two launches per step) */
    int32_t pad;
} lbpf_sp_params;

typedef struct lbpf_sp lbpf_sp;

lbpf_status lbpf_sp_workspace_size(const lbpf_sp_params* params, size_t* bytes);
lbpf_status lbpf_sp_create(const lbpf_sp_params* params, void* workspace, size_t workspace_bytes,
                           void* hip_stream, lbpf_sp** out);
/* Initial state (device arrays [ny][nx] FP32, NULL = default): a0 the density (nearly
 * incompressible, default 1) or the pressure (incompressible, default 0), u0, the source S and
 * the force (F_x, F_y) (default 0). Populations start at the equilibrium of the initial fields;
 * the histories (previous velocity, previous pressure) start at the initial fields. */
lbpf_status lbpf_sp_init(lbpf_sp* sp, const float* a0, const float* ux0, const float* uy0,
                         const float* S, const float* Fx, const float* Fy);
lbpf_status lbpf_sp_step(lbpf_sp* sp, int64_t nsteps);
/* rho (eq. 27aa; 1 in the incompressible model), u (eq. 27a) or p (rho c_s^2, or eq. 28/29)
 * of the current state into dst (device [ny][nx] FP32). Async. */
lbpf_status lbpf_sp_read(lbpf_sp* sp, int32_t field, float* dst);
/* FP64 sums over the grid of rho~ = sum_i g_i + S/2, rho u_x and rho u_y into host out[3]
 * (deterministic; synchronizes the stream). Per step the scheme changes them by exactly
 * sum S (nearly incompressible model) and sum F. */
lbpf_status lbpf_sp_sums(lbpf_sp* sp, double* out3);
int64_t lbpf_sp_step_count(const lbpf_sp* sp);
lbpf_status lbpf_sp_destroy(lbpf_sp* sp);
const char* lbpf_sp_last_error(const lbpf_sp* sp);

/* ============================================================================================
 * Three-dimensional two-phase solver on the D3Q15 lattice (Sec. 2.2, velocity matrix after
 * eq. 25: w_0 = 2/9, w_1-6 = 1/9, w_7-14 = 1/72, c_s^2 = 1/3). Same method as lbpf_ctx (eq. (24)
 * with eqs. (33), (34) at d = 3, (27a), (28) / (29); eq. (10) with eqs. (11), (14), (18); the
 * closure of Sec. 3.1; eqs. (30a)-(30b) over the fourteen D3Q15 neighbours), same conventions
 * (caller-owned device workspace, caller's stream, status codes, one host thread per handle).
 * Grids are [nz][ny][nx] with x fastest. Boundaries: fully periodic, or periodic in x and y with
 * halfway bounce-back walls half a cell below plane z = 0 and above plane z = nz - 1 (stencil
 * ghosts mirror the first fluid plane); buoyancy acts along -z: F_z = -(rho - rho_A) g.
 * ============================================================================================ */
typedef enum { LBPF3D_BC_PERIODIC = 0, LBPF3D_BC_WALLS_Z = 1 } lbpf3d_bc;

/* Fields of lbpf3d_read: phi (eq. 18), rho (eq. 3aa), u (eq. 27a), p (eq. 28 / 29), mu (eq. 8) */
typedef enum {
    LBPF3D_FIELD_PHI = 0, LBPF3D_FIELD_RHO = 1, LBPF3D_FIELD_UX = 2, LBPF3D_FIELD_UY = 3,
    LBPF3D_FIELD_UZ = 4, LBPF3D_FIELD_P = 5, LBPF3D_FIELD_MU = 6
} lbpf3d_field;

typedef struct lbpf3d_params {
    int32_t nx, ny, nz;     /* 3 <= side < 2^24 and nz * ny * pitch(nx) + 4160 < 2^30,
                             * pitch(nx) = nx rounded up to a multiple of 64 */
    int32_t variant;        /* lbpf_variant */
    int32_t pscheme;        /* lbpf_pscheme (the simplified G_0 uses d = 3) */
    int32_t fsurf;          /* lbpf_fsurf */
    int32_t visc;           /* lbpf_visc */
    int32_t bc;             /* lbpf3d_bc */
    int32_t clamp_props;    /* nonzero: phi clamped to [0,1] in rho(phi), nu(phi) */
    int32_t pad;
    double rho_A, rho_B, nu_A, nu_B, sigma, W, M_phi, tau_h; /* as in lbpf_params */
    double force_x, force_y, force_z; /* constant body-force density */
    double gravity;         /* buoyancy F_z = -(rho - rho_A) * gravity */
} lbpf3d_params;

typedef struct lbpf3d lbpf3d;

/* Bytes of device workspace: two ping-pong copies of the state (g_1..14, h_0 hi, h_1..14,
 * h_0 lo, pressure and (phi u) histories; 34 planes each, interleaved by grid row with planes
 * pitch(nx) + 32 floats apart, or as separate planes of nz * ny * pitch(nx) + 4160 floats for
 * grids too large to interleave or when the environment sets LBPF_STATE_LAYOUT=planar), then the
 * FP64 reduction area. LBPF_E_INVALID for invalid params. */
lbpf_status lbpf3d_workspace_size(const lbpf3d_params* params, size_t* bytes);
/* Validate params (as lbpf_create, plus nz) and bind a handle to a caller-owned device
 * workspace (256-byte aligned, at least lbpf3d_workspace_size bytes, else LBPF_E_NOMEM) and
 * stream. On failure *out is NULL and lbpf3d_last_error(NULL) says why. */
lbpf_status lbpf3d_create(const lbpf3d_params* params, void* workspace, size_t workspace_bytes,
                          void* hip_stream, lbpf3d** out);
/* Initial state from device arrays [nz][ny][nx] FP32 (ux, uy, uz, p may be NULL for zero):
 * h = h^eq(phi0, mu0, u0) (eq. 11, mu0 by eq. 8), g = g^eq(p0, rho(phi0), u0) (eq. 33); the
 * (phi u) and pressure histories start at phi0 u0 and p0. Resets the step count. Async. */
lbpf_status lbpf3d_init(lbpf3d* c, const float* phi, const float* ux, const float* uy,
                        const float* uz, const float* p);
/* Advance nsteps >= 0 steps, one launch each. Async. */
lbpf_status lbpf3d_step(lbpf3d* c, int64_t nsteps);
/* One lbpf3d_field of the current state into a device array [nz][ny][nx] FP32. Async. */
lbpf_status lbpf3d_read(lbpf3d* c, int32_t field, float* dst);
/* FP64 sums over the grid (sum phi of the stored h, sum rho), max |u| and the count of
 * non-finite stored values; synchronizes the stream; LBPF_E_UNSTABLE when that count is > 0. */
lbpf_status lbpf3d_diagnostics(lbpf3d* c, lbpf_diag* out);
/* Laplace-law pressure jump of Sec. 4.2 in FP64, as lbpf_laplace_dp in 3D: P = p0 - kappa phi
 * lap(phi) + kappa |grad phi|^2 / 2 + p, with the D3Q15 stencils on phi in FP64, averaged over
 * nodes within R/2 of (xc, yc, zc) minus the average over r >= R + 3W (periodic distances in
 * the periodic directions). LBPF_E_INVALID if either region is empty. Synchronizes the stream. */
lbpf_status lbpf3d_laplace_dp(lbpf3d* c, double xc, double yc, double zc, double R, double* dP);
/* Launch shapes: TX x TY tile of the x-y plane per workgroup (TX * TY threads), CZ planes per
 * chunk. Every shape gives bit-identical results. */
int32_t lbpf3d_shape_count(void);
lbpf_status lbpf3d_shape_info(int32_t shape, int32_t* tx, int32_t* ty, int32_t* cz);
lbpf_status lbpf3d_set_shape(lbpf3d* c, int32_t shape);
int32_t lbpf3d_get_shape(const lbpf3d* c);
/* Time each shape for `steps` steps and keep the fastest; *best_shape receives it. With a
 * scratch_state buffer of lbpf3d_state_size() device bytes the state and step count are saved
 * there first and restored afterwards; with NULL the state advances by the steps taken.
 * Synchronizes the stream. */
lbpf_status lbpf3d_autotune(lbpf3d* c, int32_t steps, void* scratch_state, int32_t* best_shape);
/* Checkpoint: bytes of the current state (populations, histories, step count). */
lbpf_status lbpf3d_state_size(const lbpf3d* c, size_t* bytes);
/* Copy the current state into / out of a caller device buffer of lbpf3d_state_size() bytes (a
 * 64-byte header, then the state copy as stored). A save followed by a load on another handle
 * with equal params and layout resumes bit-identically; a checkpoint of another grid or layout
 * is refused with LBPF_E_INVALID. The state copy is asynchronous on the handle's stream. */
lbpf_status lbpf3d_save_state(lbpf3d* c, void* dst_device);
lbpf_status lbpf3d_load_state(lbpf3d* c, const void* src_device);
int64_t lbpf3d_step_count(const lbpf3d* c);
lbpf_status lbpf3d_destroy(lbpf3d* c);
const char* lbpf3d_last_error(const lbpf3d* c);

#ifdef __cplusplus
}
#endif
#endif /* LBPF_H */
