/*
 * fV-SRN CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 reference of what the fV-SRN ray-march path computes
 * (Weiss, Hermueller, Westermann: "Fast Neural Representations for Direct
 * Volume Rendering"). Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library. It shares no source with the GPU
 * library: its structs, layouts and arithmetic are written here from the paper.
 *
 * All arrays are host memory, FP64, owned by the caller. Functions return 0 on
 * success and a negative value on an argument error.
 *
 * Conventions (readings of the paper where it is silent or ambiguous):
 *  - Domain [-1,1]^3. Latent grid: R vertices per axis, vertex i at
 *    -1 + 2i/(R-1) (Sec. 4.2 defines R as vertices per axis). Layout
 *    [K][z][y][x][F], channel fastest.
 *  - Network input v0 = [x, y, z, latent(F), sin-block(3L), cos-block(3L)];
 *    block entry 3k+a is sin/cos(pi * 2^k * p_a) (Eq. 1 and Eq. 2, with the
 *    frequency pi*2^k of the benchmark configuration).
 *  - Weights: for each layer i = 0..H, W_i[out][in] row-major then b_i[out].
 *    Layer 0 maps K0 = 3+F+6L -> c, layers 1..H-1 map c -> c, layer H maps
 *    c -> outputs. Layers 0..H-1 use the activation; output 0 of layer H goes
 *    through the sigmoid (Sec. 3), outputs 1..3 (when present) are the
 *    predicted density gradient in world units (Sec. 6), used as they are.
 *
 * parity pins: see tests/test_oracle_pins.py. Every function below is pinned
 * by a closed form, an invariant or brute force there; none is "parity
 * unpinned" except whole-image renders of random networks, which rest on the
 * per-stage pins.
 */
#ifndef FVSRN_ORACLE_H
#define FVSRN_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ACT_SINE = 0, ORC_ACT_SNAKEALT = 1, ORC_ACT_IDENTITY = 2 };

typedef struct {
  int32_t R, F, K;          /* latent vertices per axis, channels, keyframes */
  int32_t L;                /* Fourier octaves */
  int32_t c, H;             /* hidden width, activated layers */
  int32_t act;              /* ORC_ACT_* */
  int32_t outputs;          /* 1 (density), or 4: density logit and the predicted
                               gradient d density / d p (Sec. 6); 0 means 1 */
  const double* latent;     /* [K][R][R][R][F] */
  const double* weights;    /* packed, see header comment */
  const double* key_times;  /* [K] ascending (NULL when K == 1) */
  /* uint8 latent grid (Sec. 4.2), used instead of `latent` when non-NULL:
     vertex value = dequant[k][f][0] + dequant[k][f][1] * code[k][vertex][f] */
  const uint8_t* latent_u8;   /* [K][R][R][R][F] codes */
  const double* dequant;      /* [K][F][2] (offset, scale) */
  /* time encoding of the network input (Sec. 8): 0 latent only, 1 direct
     (the normalised time tau as one more input), 2 Fourier (sin and cos of
     pi 2^k tau, k = 0..3), 3 both; tau = 2 (clamp(t) - time_lo) /
     (time_hi - time_lo) - 1, t clamped to [time_lo, time_hi] */
  int32_t time_enc;
  int32_t pad_;
  double time_lo, time_hi;
  /* Fourier matrix (Sec. 3): [3L][3] rows of angular frequencies, the sin and
     cos blocks holding sin / cos(row . p); NULL = the octave construction
     (row 3k+a = pi 2^k e_a). Random Fourier features draw it from
     N(0, (2 pi sigma)^2). */
  const double* fourier_matrix;
} orc_net;

typedef struct {            /* piecewise-linear transfer function */
  int32_t n;                /* 2..16 control points */
  int32_t pad_;
  double density[16];       /* ascending */
  double rgba[16][4];
  double opacity_scale;     /* extinction per world unit at alpha = 1 */
} orc_tf;

typedef struct {
  int32_t ortho, width, height, pad_;
  double eye[3], target[3], up[3];
  double fov_y_deg;         /* perspective */
  double ortho_half_extent; /* orthographic: half height of the view window */
  double time;              /* keyframe time of this view */
} orc_camera;

typedef struct {
  double step;              /* world units; used when fixed_steps == 0 */
  int32_t fixed_steps;      /* > 0: that many equal segments per ray */
  int32_t phong;            /* 1: shade with the density gradient */
  double ert_eps;           /* stop once transmittance < eps (0 = never) */
  double ka, kd, ks, shininess;
  int32_t grad_fd;          /* network field: 0 = analytic (forward mode),
                               1 = central differences with step fd_step,
                               2 = the network's predicted gradient,
                               3 = reverse mode (the adjoint method) */
  int32_t pad_;
  double fd_step;
} orc_march;

/* Source of density for the renderer. */
enum { ORC_FIELD_NET = 0, ORC_FIELD_DENSE = 1, ORC_FIELD_MARSCHNER_LOBB = 2 };
typedef struct {
  int32_t kind;
  int32_t nx, ny, nz;       /* dense grid vertices per axis */
  const orc_net* net;
  const double* vol;        /* dense [nz][ny][nx] */
  double ml_fm, ml_alpha;   /* Marschner-Lobb parameters */
} orc_field;

int64_t orc_num_weights(const orc_net* net);
int32_t orc_input_width(const orc_net* net);  /* 3 + F + 6L + time inputs (0, 1, 8 or 9) */

/* Trilinear latent vector at p and keyframe time t; dz (nullable) gets
   dz[f*3+a] = d z_f / d p_a. */
int orc_latent(const orc_net* net, const double p[3], double t, double* z, double* dz);
/* Network input v0 (K0 values); dv (nullable) gets dv[j*3+a] = d v0_j / d p_a. */
int orc_features(const orc_net* net, const double p[3], double t, double* v0, double* dv);
/* Network output before the sigmoid, from an input vector. */
double orc_mlp_logit(const orc_net* net, const double* v0);
/* Density d = sigmoid(logit) at p. */
double orc_density(const orc_net* net, const double p[3], double t);
/* Density and gradient by forward-mode (tangent) propagation. */
double orc_density_grad_fwd(const orc_net* net, const double p[3], double t, double g[3]);
/* Density and gradient by reverse-mode (adjoint) propagation. */
double orc_density_grad_rev(const orc_net* net, const double p[3], double t, double g[3]);
/* Density and the gradient the network predicts (outputs 1..3; Sec. 6). */
double orc_density_grad_pred(const orc_net* net, const double p[3], double t, double g[3]);

int orc_eval_points(const orc_net* net, const double* xyz, int64_t n, double t, double* out);

/* uint8 quantisation of one keyframe grid (Sec. 4.2: per-channel minimum and
   maximum mapped to [0, 1], 8 bits), in FP32 arithmetic so that the codes are
   reproducible bit for bit: lo, hi = channel min and max; scale = (hi - lo) /
   255 (0 for a constant channel, whose codes are 0); code = round-half-even of
   (x - lo) / scale, clamped to [0, 255]. src [n][F] FP32; codes [n][F];
   dequant [F][2] = (lo, scale) as FP32 values. */
int orc_quantize_grid(const float* src, int64_t n, int32_t F, uint8_t* codes, float* dequant);
int orc_grad_points(const orc_net* net, const double* xyz, int64_t n, double t, double* out_d,
                    double* out_g);

/* Dense grid, same vertex-centred convention over [-1,1]^3. */
double orc_dense_sample(const double* vol, int nx, int ny, int nz, const double p[3]);
int orc_dense_eval_points(const double* vol, int nx, int ny, int nz, const double* xyz,
                          int64_t n, double* out);
double orc_marschner_lobb(double fm, double alpha, const double p[3], double g[3]);

/* Density and gradient of any field source (network: forward mode; dense:
   central differences with one-voxel step; Marschner-Lobb: analytic). */
double orc_field_density(const orc_field* f, const double p[3], double t, double g[3]);

int orc_tf_eval(const orc_tf* tf, double d, double rgba[4]);
/* Ray through the centre of pixel (px, py), row 0 at the top. */
int orc_camera_ray(const orc_camera* cam, int px, int py, double o[3], double dir[3]);
/* Entry/exit of the ray in [-1,1]^3; returns 0 on a miss. */
int orc_box_clip(const double o[3], const double dir[3], double* t0, double* t1);

/* Render n_views images [V][H][W][4] (premultiplied RGBA). pixels (nullable):
   list of n_pix flat indices (v*H*W + y*W + x) to render; other pixels are
   left untouched. samples (nullable) receives the number of field
   evaluations. threads <= 0: OpenMP default. */
int orc_render(const orc_field* field, const orc_tf* tf, const orc_camera* cams, int n_views,
               const orc_march* m, double* out, const int64_t* pixels, int64_t n_pix,
               int64_t* samples, int threads);

/* Structural similarity of two [H][W][4] RGBA images (the image statistic of
   Sec. 5, defined by Wang et al. 2004): per colour channel (R, G, B; alpha is
   not compared), local means, variances and covariance under an 11 x 11
   Gaussian window with sigma 1.5 (weights normalised to sum 1);
   SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
   with C1 = 0.01^2, C2 = 0.03^2 (data range 1). map [H-10][W-10] (nullable)
   gets the mean over the three channels at every pixel whose window fits;
   returns the mean of the map (or -1 on an argument error). */
double orc_ssim(const double* a, const double* b, int H, int W, double* map);

/* Adaptive resampling of the training positions (Sec. 5.4): an error grid E
   over G^3 voxels [-1,1]^3 (x fastest), per_voxel positions per voxel, and
   training positions drawn in proportion to E. Random bits are inputs: r
   holds the 32-bit outputs of a counter-based generator per point.
   orc_voxel_points: point j = v * per_voxel + s lies in voxel v at
     p_a = fma((float)i_a + u_a, 2/G, -1), u_a = (r[j][a] >> 8) 2^-24, in FP32.
   orc_error_grid: E[v] = mean over the voxel's per_voxel points of
     |density(p, t) - trilinear(vol, p)|.
   orc_weighted_points: integer weights q_v = floor(E_v * (2^24 / max E)) in
     FP32, total = sum q; point i takes the voxel v with
     Q_{v-1} <= (r[i][0] * total) >> 32 < Q_v (Q the inclusive prefix sums) and
     the position as in orc_voxel_points from r[i][1..3]. Entries that are
     not >= 0 weigh 0; with no weight at all, v = (r[i][0] * G^3) >> 32. */
int orc_voxel_points(int32_t G, int32_t per_voxel, const uint32_t* r, float* xyz);
int orc_error_grid(const orc_net* net, const double* vol, int nx, int ny, int nz, const float* xyz,
                   int64_t n_voxels, int32_t per_voxel, double t, double* E);
int orc_weighted_points(const float* E, int32_t G, int64_t n, const uint32_t* r, float* xyz);

/* Training (Sec. 3 world-space fitting; Sec. 8 for keyframe grids; Sec. 6
   for gradient-predicting networks). Gradients of
     L1 mode  (target != NULL): loss = mean_i |d(x_i, t_i) - target_i|
                 + grad_weight / 3 * mean_i sum_a |g_a(x_i, t_i) - target_grad_ia|
               (the second term only for 4-output networks with target_grad)
     VJP mode (target == NULL): loss = sum_i dloss_dd_i * d(x_i, t_i)
   with respect to all K latent grids and all weights; the gradient arrays are
   overwritten. times (nullable: all 0) gives each point's keyframe time.
   sign(0) = 0 in L1 mode. */
int orc_train_grads(const orc_net* net, const double* xyz, const double* times, int64_t n,
                    const double* target, const double* target_grad, double grad_weight,
                    const double* dloss_dd, double* d_latent, double* d_weights, double* loss);
/* One bias-corrected Adam update of n parameters at step t >= 1. */
int orc_adam(double* param, const double* grad, double* m, double* v, int64_t n, double lr,
             double beta1, double beta2, double eps, int32_t t);

#ifdef __cplusplus
}
#endif
#endif
