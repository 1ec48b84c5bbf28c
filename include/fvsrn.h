/*
 * fvsrn.h -- C ABI of the MI355X (gfx950) fV-SRN hot path.
 *
 * fV-SRN (Weiss, Hermueller, Westermann, "Fast Neural Representations for
 * Direct Volume Rendering") represents a scalar volume V: R^3 -> R as a small
 * fully connected network fed with the position, octave Fourier features of
 * the position (Sec. 3, Eq. 1 and Eq. 2) and a latent vector trilinearly
 * interpolated from a coarse grid (Sec. 4.2). Rendering evaluates the network
 * at every sample of every view ray inside one fused kernel (Sec. 4), maps the
 * predicted density through a transfer function and composites front to back.
 *
 * General rules for every entry point:
 *  - Pointers are DEVICE pointers unless marked [host]. The caller owns every
 *    buffer; the library allocates nothing and keeps no state beyond cached
 *    device properties and two static per-GPU arrays allocated with its
 *    code object: the workspace of fvsrn_train_step_noalloc and the tile
 *    counters of fvsrn_render (see there).
 *  - Device buffers must be 16-byte aligned.
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *    is the default stream). Argument errors are detected on the host before
 *    anything is launched and leave outputs untouched. Device faults surface
 *    at the caller's next synchronisation.
 *  - n == 0 (or an empty image) is a successful no-op.
 *  - Functions never throw; the status says what went wrong and
 *    fvsrn_last_error() (thread-local) gives the detail.
 *
 * Geometry and numerics (shared by every entry point):
 *  - Domain [-1,1]^3. A grid with R vertices per axis has vertex i at
 *    -1 + 2i/(R-1) (Sec. 4.2 defines R as vertices per axis); coordinates are
 *    clamped to the domain before interpolation and the cell index is capped at
 *    R-2, so p = 1 hits the last vertex exactly.
 *  - Latent grid layout [K][R_z][R_y][R_x][F]: channel fastest, then x, y, z,
 *    then keyframe.
 *  - Network input v0 = [x, y, z, latent(F), sin-block(3L), cos-block(3L),
 *    time inputs (0, 1, 8 or 9, see fvsrn_time_encoding)]; block entry 3k+a is
 *    sin / cos(pi * 2^k * p_a), k = 0..L-1 (Eq. 1 with the octave frequencies
 *    pi*2^k, Eq. 2's concatenation), unless a Fourier matrix is given.
 *  - Weights (FP32 master copy, the layout the trainer updates): for each
 *    layer i = 0..H, W_i[out][in] row-major, then b_i[out]. Layer 0 maps
 *    K0 = 3 + F + 6L (+ time inputs) inputs to c channels, layers 1..H-1 map c to c, layer H
 *    maps c to num_outputs (1, or 4 for a predicted gradient). Layers 0..H-1
 *    apply the activation (sine: sin(x); SnakeAlt: 0.5x + sin^2(x), Sec. 5
 *    Eq. 3); the sigmoid of output 0 is the density in (0,1) (Sec. 3).
 */
#ifndef FVSRN_H
#define FVSRN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FVSRN_OK = 0,
  FVSRN_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad size, misalignment, bad struct field */
  FVSRN_ERR_UNSUPPORTED = 2,      /* valid request outside the compiled configurations */
  FVSRN_ERR_WORKSPACE = 3,        /* workspace missing or too small */
  FVSRN_ERR_DEVICE = 4            /* HIP error at launch */
} fvsrn_status;

/* FVSRN_U8 is a latent-grid storage type only (uint8 codes with a per-channel
   offset and scale, Sec. 4.2). */
typedef enum { FVSRN_F32 = 0, FVSRN_F16 = 1, FVSRN_BF16 = 2, FVSRN_U8 = 3 } fvsrn_dtype;
typedef enum { FVSRN_ACT_SINE = 0, FVSRN_ACT_SNAKEALT = 1, FVSRN_ACT_IDENTITY = 2 } fvsrn_act;

/* Network and latent-grid shape (Sec. 3, Sec. 4.2). Supported: F in {8, 16},
   L in {4, 8}, c in {32, 48, 64} with 1 <= H <= 8; 2 <= R <= 512 with one
   keyframe grid (R^3 F elements) below 2^31 bytes; 1 <= K <= 64. Every
   (c, F, L) is compiled for the sine activation, the unshaded render, point
   densities and forward-mode gradients, and training for c in {32, 48}; the
   other activations, gradient modes, time encodings and Fourier matrices are
   compiled for c in {32, 48} with (F, L) = (8, 4) or (16, 8). A shape
   outside these returns FVSRN_ERR_UNSUPPORTED. */
typedef struct {
  int32_t grid_res;      /* R: latent vertices per axis */
  int32_t grid_channels; /* F: latent channels */
  int32_t grid_dtype;    /* FVSRN_F32, FVSRN_F16 or FVSRN_U8 storage of the latent grid */
  int32_t num_keyframes; /* K >= 1; K > 1 interpolates latent grids in time (Sec. 8) */
  int32_t num_freqs;     /* L: Fourier octaves */
  int32_t hidden_width;  /* c */
  int32_t hidden_layers; /* H activated layers, followed by the c -> num_outputs output layer */
  int32_t activation;    /* fvsrn_act */
  int32_t precision;     /* network arithmetic: FVSRN_F32 (FP32 MFMA), FVSRN_F16 or
                            FVSRN_BF16 (MFMA with FP32 accumulation). Phases, sigmoid,
                            TF and compositing are FP32 always; the latent
                            interpolation too, except for an FP16 or BF16 network on
                            an FP16 grid, which sums the eight corners in packed FP16
                            (its input row is rounded to FP16 or BF16 anyway). */
  int32_t num_outputs;   /* 1: the density logit; 4: the logit followed by a predicted
                            density gradient d density / d p (Sec. 6). 0 means 1. The
                            output layer holds W_out [num_outputs][c] then b_out
                            [num_outputs]; the density is the sigmoid of output 0. */
  int32_t time_encoding; /* fvsrn_time_encoding: extra network inputs from the time (Sec. 8),
                            appended to layer 0's inputs after the cosine block */
  float time_lo, time_hi; /* time range mapped onto tau in [-1, 1] (times clamped to it);
                            used when time_encoding != FVSRN_TIME_LATENT_ONLY, time_hi > time_lo */
  const float* fourier_matrix; /* [host] NULL: the octave Fourier features below. Otherwise
                            [3L][3] rows of angular frequencies (radians per world unit): the
                            sin and cos blocks hold sin / cos(row_j . p) (Sec. 3; random
                            Fourier features draw the entries from N(0, (2 pi sigma)^2)).
                            Read during the call. Built for the sine activation without a
                            time encoding: the unshaded render and point densities,
                            forward-mode gradients and Phong shading from them
                            (FP32/FP16/BF16), and training. */
} fvsrn_net_desc;

/* Time encodings (Sec. 8): the latent grids are blended in time in every case;
   DIRECT adds tau as one input, FOURIER adds sin and cos of pi 2^k tau for
   k = 0..3 (8 inputs), BOTH adds tau then the 8 Fourier inputs. Networks with a
   time input are built for the sine activation: the unshaded render and point
   densities, forward-mode gradients and Phong shading from them
   (FP32/FP16/BF16; the time inputs have no position derivative), and
   training. */
typedef enum {
  FVSRN_TIME_LATENT_ONLY = 0,
  FVSRN_TIME_DIRECT = 1,
  FVSRN_TIME_FOURIER = 2,
  FVSRN_TIME_BOTH = 3
} fvsrn_time_encoding;

typedef struct {
  const void* latent;       /* [K][R][R][R][F] in grid_dtype */
  const float* weights;     /* FP32 packed weights (layout above) */
  const float* key_times;   /* [host] [K] strictly ascending keyframe times; NULL if K == 1.
                               A time t is clamped to [key_times[0], key_times[K-1]] and the
                               two neighbouring keyframe latents are blended linearly. */
  const float* latent_dequant; /* FVSRN_U8 grids: device [K][F][2] (offset, scale); vertex
                               value = offset + scale * code (fvsrn_quantize_grid makes both).
                               Ignored for other grid types. */
} fvsrn_params;

/* [host] Piecewise-linear transfer function: density -> (r, g, b, alpha),
   constant beyond the first and last control point. Extinction per world
   unit is opacity_scale * alpha. 2 <= n <= 16, densities strictly ascending. */
typedef struct {
  int32_t n;
  float density[16];
  float rgba[16][4];
  float opacity_scale;
} fvsrn_tf;

/* [host] Look-at camera. forward = normalize(target - eye),
   right = normalize(forward x up), true up = right x forward. Pixel (x, y),
   row 0 at the top, has NDC ((2x+1)/W - 1, 1 - (2y+1)/H). Perspective rays
   start at eye with direction forward + tan(fov_y/2)(aspect ndc_x right +
   ndc_y up); orthographic rays start at eye + h(aspect ndc_x right + ndc_y up)
   with direction forward, h = ortho_half_extent. `time` selects the keyframe
   blend of this view. */
typedef struct {
  int32_t ortho;
  float eye[3], target[3], up[3];
  float fov_y_deg, ortho_half_extent;
  int32_t width, height;
  float time;
} fvsrn_camera;

/* [host] Ray-march settings. The ray's chord [t0, t1] inside [-1,1]^3
   (t0 >= 0) is cut into fixed_steps equal segments (fixed_steps > 0), else
   into segments of length `step` with the last one clipped at t1. Each
   segment is sampled at its midpoint. With extinction kappa and length ds:
   a = 1 - exp(-kappa ds), C += T a rgb, A += T a, T *= exp(-kappa ds); the
   march stops after a sample once T < ert_eps (0 disables early ray
   termination). phong != 0 shades rgb with a headlight Blinn-Phong term from
   the normalized density gradient n: rgb (ka + kd |n.l|) + ks |n.l|^shininess
   (Sec. 6), gradients below 1e-6 in length leave rgb unshaded; ka, kd, ks
   and shininess must be finite, non-negative and at most 1e6. For the
   network, grad_mode selects how the gradient is obtained (Sec. 6):
   FVSRN_GRAD_FORWARD differentiates the network in forward mode;
   FVSRN_GRAD_CENTRAL takes central differences of the network density with
   step fd_step (> 0, world units): seven network evaluations per sample;
   FVSRN_GRAD_PREDICTED uses outputs 1..3 of a num_outputs == 4 network as the
   gradient (one evaluation per sample, no differentiation);
   FVSRN_GRAD_ADJOINT backpropagates through the network to the position
   (reverse mode: one forward and one transposed pass per sample).
   Dense-grid rendering always uses one-voxel central differences. */
typedef enum {
  FVSRN_GRAD_FORWARD = 0,
  FVSRN_GRAD_CENTRAL = 1,
  FVSRN_GRAD_PREDICTED = 2,
  FVSRN_GRAD_ADJOINT = 3
} fvsrn_grad_mode;
typedef struct {
  float step;
  int32_t fixed_steps;
  float ert_eps;
  int32_t phong;
  float ka, kd, ks, shininess;
  int32_t grad_mode;
  float fd_step;
} fvsrn_march;

/* Render n_views images of the fV-SRN with one launch (Sec. 4, Sec. 5.1):
   out_rgba [n_views][H][W][4] FP32, premultiplied colour and opacity over a
   transparent background. All cameras must share width and height.
   stats (nullable, device, 3 x u64, accumulated -- the caller zeroes it):
   [0] += samples composited, [1] += rays that hit the domain, [2] += sample
   slots issued (rays per wave x march steps of the wave, idle rays included;
   [0]/[2] is the occupancy of the matrix tiles). A wave marches 64 rays
   without shading, 16 with forward-mode gradients and 8 with central
   differences. Phong shading needs the density gradient, obtained as
   march->grad_mode selects (Sec. 6), for FP32, FP16 and BF16 networks
   (central differences and predicted gradients for the sine activation,
   also with a time encoding or a Fourier matrix; the adjoint for the sine
   activation with the octave Fourier features and no time input; the
   adjoint of an FP32 network whose weight fragments, forward and transposed,
   exceed the 160 KiB of LDS -- c = 48 with H = 8, or with F = 16 and H >= 7 --
   is not available); other combinations return FVSRN_ERR_UNSUPPORTED.
   Predicted gradients need num_outputs == 4.
   Each launch is persistent (as many workgroups as the GPU holds at once)
   and hands its tiles out through a pair of counters in a static per-GPU
   array of 1024 pairs; successive calls on a device take successive pairs,
   so at most 1024 fvsrn_render launches (one per 16 views of a call)
   may be in flight on one GPU at once. */
fvsrn_status fvsrn_render(const fvsrn_net_desc* desc, const fvsrn_params* params,
                          const fvsrn_tf* tf, const fvsrn_camera* cams, int32_t n_views,
                          const fvsrn_march* march, float* out_rgba,
                          unsigned long long* stats, void* stream);

/* Density of the fV-SRN at n arbitrary points (Sec. 3: each position is
   evaluated independently; Sec. 7 times 10^6 random reconstructions).
   xyz [n][3] FP32, out_density [n] FP32; time selects the keyframe blend. */
fvsrn_status fvsrn_eval_points(const fvsrn_net_desc* desc, const fvsrn_params* params,
                               const float* xyz, int64_t n, float time, float* out_density,
                               void* stream);

/* Density and its gradient d density / d p at n points (Sec. 6), by
   grad_mode: FVSRN_GRAD_FORWARD differentiates through the network, the
   Fourier features and the trilinear interpolation in forward mode;
   FVSRN_GRAD_ADJOINT does the same in reverse mode (same availability as in
   fvsrn_render); FVSRN_GRAD_PREDICTED returns outputs 1..3 of a
   num_outputs == 4 network (one plain evaluation). FVSRN_GRAD_CENTRAL is not
   offered here. out_density nullable [n]; out_grad [n][3]. */
fvsrn_status fvsrn_grad_points(const fvsrn_net_desc* desc, const fvsrn_params* params,
                               const float* xyz, int64_t n, float time, int32_t grad_mode,
                               float* out_density, float* out_grad, void* stream);

/* [host] Adam state for fvsrn_train_step (bias-corrected; PyTorch's form
   p -= lr/(1-b1^t) * m / (sqrt(v)/sqrt(1-b2^t) + eps)). */
typedef struct {
  float lr_grid, lr_mlp, beta1, beta2, eps;
  int32_t step;          /* t >= 1 of this update */
  float* m_latent;       /* device [K R^3 F] */
  float* v_latent;
  float* m_weights;      /* device [n_weights] */
  float* v_weights;
} fvsrn_adam;

/* One world-space training step on n points (Sec. 3, Sec. 5: L1 loss, Adam;
   Sec. 8 for keyframe grids). FP32 latent grids and FP32 weights (the master
   copy), FP32 gradients and Adam. desc->precision selects the network's
   arithmetic: FVSRN_F32 (FP32 MFMA), or FVSRN_F16 -- forward and backward on
   FP16 MFMA with FP32 accumulation, the forward pass identical to the FP16
   render's, dL/dy scaled by 2^floor(log2 n) before it is rounded to FP16 and
   every gradient by the inverse power of two; built for L1 mode, the sine,
   SnakeAlt and identity activations, c in {32, 48} with (F, L) = (8, 4) or
   (16, 8), no time input or Fourier matrix (other FP16 requests return
   FVSRN_ERR_UNSUPPORTED).
     L1 mode  (target != NULL): loss = mean |d(x_i, t_i) - target_i|, sign(0) = 0.
       For a num_outputs == 4 network with target_grad != NULL ([n][3]) the
       predicted gradient g_i (outputs 1..3) is fitted as well (Sec. 6):
       loss += grad_weight / 3 * mean sum_a |g_i,a - target_grad_i,a|.
     VJP mode (target == NULL): loss = sum dloss_dy_i * d(x_i, t_i) (the
       gradient of any downstream loss, e.g. from autograd).
   latent [K][R^3 F]; key_times [host, K] strictly ascending (NULL when
   K == 1); times (device [n], nullable: all 0) is each point's time, which
   blends the two neighbouring keyframes as in rendering, so a point's latent
   gradient goes to both with the blend weights.
   d_latent [K R^3 F] and d_weights [n_weights] are overwritten with the
   gradients (d_weights bitwise reproducible; d_latent gathered per vertex
   over the points of its eight cells after a counting sort of the points by
   cell (for a single keyframe summed per cell and corner first), whose order
   within a cell may vary between calls, so d_latent is reproducible to
   rounding). n < 2^31. With adam != NULL the latent grids and the weights are then
   updated in place (lr_grid for the latent grids, lr_mlp for the weights).
   out_loss (nullable, device FP32 scalar) receives the loss. workspace
   (16-byte aligned) must hold fvsrn_train_workspace_size(desc, n) bytes. */
fvsrn_status fvsrn_train_step(const fvsrn_net_desc* desc, float* latent, float* weights,
                              const float* key_times, float* d_latent, float* d_weights,
                              const float* xyz, const float* times, int64_t n,
                              const float* target, const float* target_grad, float grad_weight,
                              const float* dloss_dy, const fvsrn_adam* adam, float* out_loss, void* workspace,
                              size_t workspace_bytes, void* stream);
size_t fvsrn_train_workspace_size(const fvsrn_net_desc* desc, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving or training loops, harnesses that forbid
   hipMalloc): fvsrn_train_step with the same arguments, minus the
   workspace, and the same results (the same kernels and partition, so
   d_weights equals fvsrn_train_step's bit for bit). It allocates nothing:
   its workspace is a static device array of FVSRN_TRAIN_STATIC_WORKSPACE_BYTES
   on each GPU, allocated with the library's code object and held until the
   process ends. A step whose fvsrn_train_workspace_size exceeds that returns
   FVSRN_ERR_WORKSPACE before any launch (e.g. 2^18 points fit the 32^3 x 16,
   4 x 32 network, 82 MiB, and the 64^3 x 16, 4 x 48 one, 76 MiB; 3 x 2^18
   points on the latter, 114 MiB, do not).
   Every call on one GPU shares that GPU's array and the kernels overwrite
   or clear what they use, so calls that overlap on one GPU (other streams,
   other host threads) race and must be serialised by the caller. The
   device address is looked up once per GPU at the first call on it. */
#define FVSRN_TRAIN_STATIC_WORKSPACE_BYTES ((size_t)96 << 20)
fvsrn_status fvsrn_train_step_noalloc(const fvsrn_net_desc* desc, float* latent, float* weights,
                                      const float* key_times, float* d_latent, float* d_weights,
                                      const float* xyz, const float* times, int64_t n,
                                      const float* target, const float* target_grad, float grad_weight,
                                      const float* dloss_dy, const fvsrn_adam* adam, float* out_loss,
                                      void* stream);

/* Plain dense-grid DVR with the same rays, transfer function and compositor
   (the uncompressed reference the paper renders, Sec. 5): vol [nz][ny][nx]
   FP32, vertex-centred over [-1,1]^3, trilinear lookup. Phong uses central
   differences with a one-voxel step (Sec. 6). stats as for fvsrn_render
   ([2] counts one slot per composited sample). */
fvsrn_status fvsrn_render_dense(const float* vol, int32_t nx, int32_t ny, int32_t nz,
                                const fvsrn_tf* tf, const fvsrn_camera* cams, int32_t n_views,
                                const fvsrn_march* march, float* out_rgba,
                                unsigned long long* stats, void* stream);

/* Trilinear samples of a dense grid at n points (training targets drawn from
   the original volume, Sec. 3). */
fvsrn_status fvsrn_dense_eval_points(const float* vol, int32_t nx, int32_t ny, int32_t nz,
                                     const float* xyz, int64_t n, float* out, void* stream);

/* Trilinear samples and their gradient by central differences with a
   one-voxel step per axis (2 / (n_axis - 1) world units, as the dense
   renderer shades, Sec. 6): the gradient targets of predicted-gradient
   training. out_density nullable [n]; out_grad [n][3]. */
fvsrn_status fvsrn_dense_grad_points(const float* vol, int32_t nx, int32_t ny, int32_t nz,
                                     const float* xyz, int64_t n, float* out_density,
                                     float* out_grad, void* stream);

/* n uniform points in [-1,1)^3 from a Philox4x32-10 counter-based generator
   (Salmon et al., SC'11): point i uses counter (i mod 2^32, i div 2^32,
   counter_lo, counter_hi) and key (seed_lo, seed_hi); its three coordinates come from the first three
   32-bit outputs u as -1 + (u >> 8) * 2^-23. xyz [n][3]. */
fvsrn_status fvsrn_sample_points(uint64_t seed, uint64_t counter, int64_t n, float* xyz,
                                 void* stream);

/* Adaptive resampling of training positions (Sec. 5.4: every N epochs an
   error grid over G^3 voxels, a few positions per voxel, then new training
   positions in proportion to the error). Voxel v = (ix, iy, iz), x fastest,
   spans [-1 + 2 i_a / G, -1 + 2 (i_a + 1) / G] per axis. Random words come
   from Philox4x32-10 as in fvsrn_sample_points; a position inside voxel v
   from words r_a is p_a = fma((float)i_a + (r_a >> 8) 2^-24, 2/G, -1) in FP32.

   fvsrn_voxel_points: point j = v * per_voxel + s of the G^3 * per_voxel
   error-grid points (counter j, words 0..2). xyz [G^3 per_voxel][3];
   G^3 * per_voxel < 2^32. */
fvsrn_status fvsrn_voxel_points(uint64_t seed, uint64_t counter, int32_t G, int32_t per_voxel, float* xyz,
                                void* stream);

/* E[v] = mean over voxel v's per_voxel points xyz[v per_voxel + s] of
   |fV-SRN density(p, time) - trilinear(vol, p)| (vol [nz][ny][nx] FP32, the
   training target). scratch: n_voxels * per_voxel floats (device) for the
   network densities. E [n_voxels] FP32. FP32 networks. */
fvsrn_status fvsrn_error_grid(const fvsrn_net_desc* desc, const fvsrn_params* params, const float* vol,
                              int32_t nx, int32_t ny, int32_t nz, const float* xyz, int64_t n_voxels,
                              int32_t per_voxel, float time, float* E, float* scratch, void* stream);

/* n training positions drawn in proportion to the error grid E [G^3]
   (device FP32): integer weights q_v = floor(E_v * (2^24 / max E)) (FP32
   arithmetic; entries that are not >= 0 weigh 0), Q their inclusive prefix
   sums; point i (counter i) takes the voxel v with
   Q_{v-1} <= (r_0 * Q_{G^3-1}) >> 32 < Q_v (with no weight at all,
   v = (r_0 G^3) >> 32) and its position from words 1..3. workspace: device,
   fvsrn_weighted_points_workspace_size(G) bytes; it keeps Q after the call.
   E == NULL draws from the Q already in the workspace (left there by an
   earlier call with the same G and an error grid, unchanged since): the
   same positions as passing that grid again, without rebuilding Q -- for
   the steps between two refreshes of the error grid. */
fvsrn_status fvsrn_sample_points_weighted(uint64_t seed, uint64_t counter, const float* E, int32_t G, int64_t n,
                                          float* xyz, void* workspace, size_t workspace_bytes, void* stream);

/* The draws of n_grids calls of fvsrn_sample_points_weighted with E == NULL,
   in one launch: for a batch taken from several error grids (one per
   timestep of a time-varying volume, Sec. 5.4 with Sec. 8), where separate
   calls would each cost a launch. Grid k draws n_per_grid[k] points (host
   array, each in [0, 2^40]) with counter + k from the prefix sums in
   workspace slice k (workspace + k * workspace_stride bytes, left there by
   an earlier fvsrn_sample_points_weighted call with the same G and that
   grid's E), written to xyz + 3 (n_per_grid[0] + ... + n_per_grid[k-1]):
   the same positions as those n_grids calls. 1 <= n_grids <= 64;
   workspace and workspace_stride 16-byte aligned, the stride at least
   fvsrn_weighted_points_workspace_size(G); xyz [sum n_per_grid][3]. */
fvsrn_status fvsrn_sample_points_weighted_multi(uint64_t seed, uint64_t counter, int32_t G, int32_t n_grids,
                                                const int64_t* n_per_grid, float* xyz, const void* workspace,
                                                size_t workspace_stride, void* stream);
size_t fvsrn_weighted_points_workspace_size(int32_t G);

/* Round an FP32 array to FP16 or BF16 (round to nearest even), e.g. to store
   the latent grid in FP16. dst_dtype FVSRN_F16 or FVSRN_BF16. */
fvsrn_status fvsrn_cast_grid(const float* src, void* dst, int64_t count, int32_t dst_dtype,
                             void* stream);

/* uint8 quantisation of one keyframe grid (Sec. 4.2: per channel, the
   minimum and maximum are mapped to [0, 1] and stored in 8 bits). src
   [n_vertices][channels] FP32 (device); codes [n_vertices][channels] uint8;
   dequant [channels][2] = (lo, scale) FP32 with scale = (hi - lo) / 255 and
   code = round-half-even((x - lo) / scale) clamped to [0, 255] (0 when a
   channel is constant), all in FP32 arithmetic. For K keyframes call it once
   per keyframe with the pointers advanced. 1 <= channels <= 64. */
fvsrn_status fvsrn_quantize_grid(const float* src, int64_t n_vertices, int32_t channels, uint8_t* codes,
                                 float* dequant, void* stream);

/* Structural similarity map of image pairs (the image statistic of Sec. 5,
   defined by Wang et al. 2004): a, b [n_images][height][width][4] RGBA FP32
   (device); per colour channel (R, G, B), Gaussian-window statistics (11 x 11,
   sigma 1.5, normalised) give
   ((2 mu_a mu_b + C1)(2 s_ab + C2)) / ((mu_a^2 + mu_b^2 + C1)(s_a^2 + s_b^2 + C2)),
   C1 = 0.01^2, C2 = 0.03^2 (data range 1); out_map [n_images][height-10][width-10]
   (device) receives its mean over the three channels at every pixel whose
   window fits. The SSIM of an image is the mean of its map. width, height >= 11. */
fvsrn_status fvsrn_ssim_map(const float* a, const float* b, int32_t width, int32_t height, int32_t n_images,
                            float* out_map, void* stream);

/* Number of FP32 weights of a network description (0 if invalid). */
int64_t fvsrn_num_weights(const fvsrn_net_desc* desc);

const char* fvsrn_status_str(fvsrn_status s);
const char* fvsrn_last_error(void); /* thread-local detail of the last failing call */

/* SHA-256 (hex) of the sources this library was built from (this header and
   the HIP/C++ sources), so that a caller can refuse a library that is older
   than the sources next to it. Static string, never NULL. */
const char* fvsrn_build_id(void);

#ifdef __cplusplus
}
#endif
#endif /* FVSRN_H */
