/*
 * fV-SRN CPU oracle -- TEST INFRASTRUCTURE ONLY (see fvsrn_oracle.h).
 *
 * Plain FP64 loops, one function per step of the method, in the order the
 * paper describes them. No blocking, fusion or reordering: each function can be
 * checked against its section by eye. Built with gcc, no fast-math.
 */
#include "fvsrn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- layout */

/* Input width of the first layer: position (3), latent vector (F) and the
   sine and cosine Fourier blocks (3L each) -- Sec. 3 Eq. 2 and Sec. 4.2. */
/* Time inputs by encoding (Sec. 8): none, tau, four sin/cos octaves of tau, both. */
static int time_inputs(const orc_net* net) {
  static const int n[4] = {0, 1, 8, 9};
  return (net->time_enc >= 0 && net->time_enc < 4) ? n[net->time_enc] : 0;
}

int32_t orc_input_width(const orc_net* net) { return 3 + net->F + 6 * net->L + time_inputs(net); }

static int layer_in(const orc_net* net, int i) { return i == 0 ? orc_input_width(net) : net->c; }
static int n_outputs(const orc_net* net) { return net->outputs > 1 ? net->outputs : 1; }
static int layer_out(const orc_net* net, int i) { return i == net->H ? n_outputs(net) : net->c; }

/* Offset of W_i in the packed weight array; b_i follows W_i. */
static int64_t layer_offset(const orc_net* net, int i) {
  int64_t off = 0;
  for (int j = 0; j < i; ++j) off += (int64_t)layer_out(net, j) * layer_in(net, j) + layer_out(net, j);
  return off;
}

int64_t orc_num_weights(const orc_net* net) { return layer_offset(net, net->H + 1); }

static int net_ok(const orc_net* net) {
  return net && net->R >= 2 && net->F >= 0 && net->K >= 1 && net->L >= 0 && net->c >= 1 &&
         (net->outputs <= 1 || net->outputs == 4) &&
         net->H >= 1 && net->weights && (net->F == 0 || net->latent || (net->latent_u8 && net->dequant)) &&
         (net->K == 1 || net->key_times) && net->time_enc >= 0 && net->time_enc < 4 &&
         (net->time_enc == 0 || net->time_hi > net->time_lo);
}

/* ------------------------------------------------------- latent grid (4.2) */

/* Grid coordinate along one axis: vertex i sits at -1 + 2i/(R-1). Positions
   outside [-1,1] are clamped (their derivative is then zero); the cell index
   is capped at R-2 so that p = 1 lands on the last vertex of the last cell. */
static void axis_cell(double p, int R, int* i0, double* frac, double* dfrac_dp) {
  double u = (p + 1.0) * 0.5 * (double)(R - 1);
  double du = 0.5 * (double)(R - 1);
  if (u <= 0.0) { u = 0.0; if (p < -1.0) du = 0.0; }
  if (u >= (double)(R - 1)) { u = (double)(R - 1); if (p > 1.0) du = 0.0; }
  int i = (int)floor(u);
  if (i > R - 2) i = R - 2;
  *i0 = i;
  *frac = u - (double)i;
  *dfrac_dp = du;
}

/* Trilinear interpolation of one keyframe grid: z = sum over the 8 cell
   corners of w_corner * G[corner] (Sec. 4.2). */
static void latent_one(const orc_net* net, int key, const double p[3], double* z, double* dz) {
  const int R = net->R, F = net->F;
  int i[3];
  double f[3], df[3];
  for (int a = 0; a < 3; ++a) axis_cell(p[a], R, &i[a], &f[a], &df[a]);
  for (int ch = 0; ch < F; ++ch) {
    z[ch] = 0.0;
    if (dz) dz[ch * 3 + 0] = dz[ch * 3 + 1] = dz[ch * 3 + 2] = 0.0;
  }
  const int64_t kbase = (int64_t)key * R * R * R * F;
  const double* G = net->latent_u8 ? NULL : net->latent + kbase;
  const uint8_t* Gq = net->latent_u8 ? net->latent_u8 + kbase : NULL;
  const double* dq = net->latent_u8 ? net->dequant + (int64_t)key * F * 2 : NULL;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        double wx = cx ? f[0] : 1.0 - f[0];
        double wy = cy ? f[1] : 1.0 - f[1];
        double wz = cz ? f[2] : 1.0 - f[2];
        double dwx = (cx ? 1.0 : -1.0) * df[0];
        double dwy = (cy ? 1.0 : -1.0) * df[1];
        double dwz = (cz ? 1.0 : -1.0) * df[2];
        const int64_t v = (((int64_t)(i[2] + cz) * R + (i[1] + cy)) * R + (i[0] + cx)) * F;
        for (int ch = 0; ch < F; ++ch) {
          /* the vertex value: stored, or de-quantised from its code */
          const double g = G ? G[v + ch] : dq[2 * ch] + dq[2 * ch + 1] * (double)Gq[v + ch];
          z[ch] += wx * wy * wz * g;
          if (dz) {
            dz[ch * 3 + 0] += dwx * wy * wz * g;
            dz[ch * 3 + 1] += wx * dwy * wz * g;
            dz[ch * 3 + 2] += wx * wy * dwz * g;
          }
        }
      }
}

/* Keyframe selection for time t (Sec. 8): clamp t to the keyframe range and
   interpolate linearly between the two neighbouring keyframes. */
static void key_pair(const orc_net* net, double t, int* k, double* w) {
  if (net->K == 1) { *k = 0; *w = 0.0; return; }
  const double* kt = net->key_times;
  if (t <= kt[0]) { *k = 0; *w = 0.0; return; }
  if (t >= kt[net->K - 1]) { *k = net->K - 2; *w = 1.0; return; }
  int j = 0;
  while (j + 1 < net->K - 1 && kt[j + 1] <= t) ++j;
  *k = j;
  *w = (t - kt[j]) / (kt[j + 1] - kt[j]);
}

int orc_latent(const orc_net* net, const double p[3], double t, double* z, double* dz) {
  if (!net_ok(net) || !z) return -1;
  const int F = net->F;
  int k;
  double w;
  key_pair(net, t, &k, &w);
  latent_one(net, k, p, z, dz);
  if (net->K > 1) {
    double* z1 = (double*)malloc(sizeof(double) * (size_t)F * 4);
    double* dz1 = z1 + F;
    latent_one(net, k + 1, p, z1, dz ? dz1 : NULL);
    for (int ch = 0; ch < F; ++ch) {
      z[ch] = (1.0 - w) * z[ch] + w * z1[ch];
      if (dz)
        for (int a = 0; a < 3; ++a) dz[ch * 3 + a] = (1.0 - w) * dz[ch * 3 + a] + w * dz1[ch * 3 + a];
    }
    free(z1);
  }
  return 0;
}

/* ----------------------------------------------- network input (Sec. 3) */

/* v0 = p (+) z (+) sin(F p) (+) cos(F p) with the Fourier matrix rows ordered
   octave-major: row 3k+a has frequency pi*2^k on axis a (Eq. 1, Eq. 2), or
   the rows of a given matrix (random Fourier features). */
int orc_features(const orc_net* net, const double p[3], double t, double* v0, double* dv) {
  if (!net_ok(net) || !v0) return -1;
  const int F = net->F, L = net->L, K0 = orc_input_width(net);
  if (dv) memset(dv, 0, sizeof(double) * (size_t)K0 * 3);
  for (int a = 0; a < 3; ++a) {
    v0[a] = p[a];
    if (dv) dv[a * 3 + a] = 1.0;
  }
  if (F > 0) {
    double* dz = dv ? (double*)malloc(sizeof(double) * (size_t)F * 3) : NULL;
    orc_latent(net, p, t, v0 + 3, dz);
    if (dv)
      for (int ch = 0; ch < F; ++ch)
        for (int a = 0; a < 3; ++a) dv[(3 + ch) * 3 + a] = dz[ch * 3 + a];
    free(dz);
  }
  const int s0 = 3 + F, c0 = 3 + F + 3 * L;
  if (net->fourier_matrix) {
    /* a general Fourier matrix: phase_j = F_j . p, d phase_j / d p_a = F_ja */
    for (int j = 0; j < 3 * L; ++j) {
      const double* fj = net->fourier_matrix + 3 * j;
      double ph = fj[0] * p[0] + fj[1] * p[1] + fj[2] * p[2];
      v0[s0 + j] = sin(ph);
      v0[c0 + j] = cos(ph);
      if (dv)
        for (int a = 0; a < 3; ++a) {
          dv[(s0 + j) * 3 + a] = fj[a] * cos(ph);
          dv[(c0 + j) * 3 + a] = -fj[a] * sin(ph);
        }
    }
  } else {
    for (int k = 0; k < L; ++k)
      for (int a = 0; a < 3; ++a) {
        double freq = M_PI * ldexp(1.0, k);
        v0[s0 + 3 * k + a] = sin(freq * p[a]);
        v0[c0 + 3 * k + a] = cos(freq * p[a]);
        if (dv) {
          dv[(s0 + 3 * k + a) * 3 + a] = freq * cos(freq * p[a]);
          dv[(c0 + 3 * k + a) * 3 + a] = -freq * sin(freq * p[a]);
        }
      }
  }
  /* time inputs (Sec. 8), after the spatial Fourier block; they do not
     depend on p */
  if (net->time_enc != 0) {
    double tc = t < net->time_lo ? net->time_lo : (t > net->time_hi ? net->time_hi : t);
    double tau = 2.0 * (tc - net->time_lo) / (net->time_hi - net->time_lo) - 1.0;
    int j = 3 + F + 6 * L;
    if (net->time_enc == 1 || net->time_enc == 3) v0[j++] = tau;
    if (net->time_enc >= 2) {
      for (int k = 0; k < 4; ++k) v0[j + k] = sin(M_PI * ldexp(1.0, k) * tau);
      for (int k = 0; k < 4; ++k) v0[j + 4 + k] = cos(M_PI * ldexp(1.0, k) * tau);
    }
  }
  return 0;
}

/* ------------------------------------------------ the MLP (Sec. 3, Eq. 3) */

static double act_f(int act, double x) {
  switch (act) {
    case ORC_ACT_SINE: return sin(x);
    case ORC_ACT_SNAKEALT: return 0.5 * x + sin(x) * sin(x); /* Eq. 3 */
    default: return x;
  }
}

static double act_df(int act, double x) {
  switch (act) {
    case ORC_ACT_SINE: return cos(x);
    case ORC_ACT_SNAKEALT: return 0.5 + 2.0 * sin(x) * cos(x);
    default: return 1.0;
  }
}

static double sigmoid(double y) { return 1.0 / (1.0 + exp(-y)); }

/* v_{i+1} = a(W_i v_i + b_i) for the H activated layers, then the output
   layer without activation (the density's sigmoid is applied by the caller).
   Keeps the pre-activations a_i (H*c values) when pre != NULL and the last
   hidden layer's output when hlast != NULL; writes all outputs to y (when
   non-NULL) and returns output 0, the density logit. */
static double mlp_outputs(const orc_net* net, const double* v0, double* pre, double* hlast, double* y) {
  const int c = net->c, H = net->H;
  int width = orc_input_width(net);
  double* h = (double*)malloc(sizeof(double) * (size_t)(width > c ? width : c) * 2);
  double* hn = h + (width > c ? width : c);
  memcpy(h, v0, sizeof(double) * (size_t)width);
  for (int i = 0; i < H; ++i) {
    const double* W = net->weights + layer_offset(net, i);
    const double* b = W + (int64_t)c * width;
    for (int j = 0; j < c; ++j) {
      double s = b[j];
      for (int k = 0; k < width; ++k) s += W[(int64_t)j * width + k] * h[k];
      if (pre) pre[i * c + j] = s;
      hn[j] = act_f(net->act, s);
    }
    memcpy(h, hn, sizeof(double) * (size_t)c);
    width = c;
  }
  const int no = n_outputs(net);
  const double* W = net->weights + layer_offset(net, H);
  double y0 = 0.0;
  for (int j = 0; j < no; ++j) {
    double s = W[(int64_t)no * c + j];
    for (int k = 0; k < c; ++k) s += W[(int64_t)j * c + k] * h[k];
    if (y) y[j] = s;
    if (j == 0) y0 = s;
  }
  if (hlast) memcpy(hlast, h, sizeof(double) * (size_t)c);
  free(h);
  return y0;
}

static double mlp_forward(const orc_net* net, const double* v0, double* pre) {
  return mlp_outputs(net, v0, pre, NULL, NULL);
}

double orc_mlp_logit(const orc_net* net, const double* v0) {
  if (!net_ok(net) || !v0) return NAN;
  return mlp_forward(net, v0, NULL);
}

double orc_density(const orc_net* net, const double p[3], double t) {
  if (!net_ok(net)) return NAN;
  double* v0 = (double*)malloc(sizeof(double) * (size_t)orc_input_width(net));
  orc_features(net, p, t, v0, NULL);
  double d = sigmoid(mlp_forward(net, v0, NULL));
  free(v0);
  return d;
}

/* Forward mode: push the three tangent columns d v0 / d p through every
   layer alongside the values (chain rule layer by layer). */
double orc_density_grad_fwd(const orc_net* net, const double p[3], double t, double g[3]) {
  if (!net_ok(net) || !g) return NAN;
  const int c = net->c, H = net->H, K0 = orc_input_width(net);
  const int mx = K0 > c ? K0 : c;
  double* h = (double*)malloc(sizeof(double) * (size_t)mx * 8);
  double* th = h + mx;           /* [mx][3] */
  double* hn = th + 3 * mx;      /* [mx] */
  double* thn = hn + mx;         /* [mx][3] */
  orc_features(net, p, t, h, th);
  int width = K0;
  for (int i = 0; i < H; ++i) {
    const double* W = net->weights + layer_offset(net, i);
    const double* b = W + (int64_t)c * width;
    for (int j = 0; j < c; ++j) {
      double s = b[j], ts[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < width; ++k) {
        double w = W[(int64_t)j * width + k];
        s += w * h[k];
        for (int a = 0; a < 3; ++a) ts[a] += w * th[k * 3 + a];
      }
      hn[j] = act_f(net->act, s);
      double da = act_df(net->act, s);
      for (int a = 0; a < 3; ++a) thn[j * 3 + a] = da * ts[a];
    }
    memcpy(h, hn, sizeof(double) * (size_t)c);
    memcpy(th, thn, sizeof(double) * (size_t)c * 3);
    width = c;
  }
  const double* W = net->weights + layer_offset(net, H);
  double y = W[(int64_t)n_outputs(net) * c], ty[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < c; ++k) {
    y += W[k] * h[k];
    for (int a = 0; a < 3; ++a) ty[a] += W[k] * th[k * 3 + a];
  }
  double d = sigmoid(y);
  for (int a = 0; a < 3; ++a) g[a] = d * (1.0 - d) * ty[a];
  free(h);
  return d;
}

/* Reverse mode (the adjoint method of Sec. 6): one forward pass keeping the
   pre-activations, then the transposed layers back to d v0, then the chain
   rule through the input features. */
double orc_density_grad_rev(const orc_net* net, const double p[3], double t, double g[3]) {
  if (!net_ok(net) || !g) return NAN;
  const int c = net->c, H = net->H, K0 = orc_input_width(net);
  const int mx = K0 > c ? K0 : c;
  double* v0 = (double*)malloc(sizeof(double) * ((size_t)K0 * 4 + (size_t)H * c + 2 * (size_t)mx));
  double* dv = v0 + K0;          /* [K0][3] */
  double* pre = dv + 3 * K0;     /* [H][c] */
  double* delta = pre + (size_t)H * c;
  double* dnext = delta + mx;
  orc_features(net, p, t, v0, dv);
  double d = sigmoid(mlp_forward(net, v0, pre));
  const double* Wout = net->weights + layer_offset(net, H);
  for (int k = 0; k < c; ++k) delta[k] = d * (1.0 - d) * Wout[k]; /* d d / d h_H */
  for (int i = H - 1; i >= 0; --i) {
    const int width = layer_in(net, i);
    const double* W = net->weights + layer_offset(net, i);
    for (int j = 0; j < c; ++j) delta[j] *= act_df(net->act, pre[i * c + j]);
    for (int k = 0; k < width; ++k) {
      double s = 0.0;
      for (int j = 0; j < c; ++j) s += W[(int64_t)j * width + k] * delta[j];
      dnext[k] = s;
    }
    memcpy(delta, dnext, sizeof(double) * (size_t)width);
  }
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
    for (int k = 0; k < K0; ++k) s += delta[k] * dv[k * 3 + a];
    g[a] = s;
  }
  free(v0);
  return d;
}

double orc_density_grad_pred(const orc_net* net, const double p[3], double t, double g[3]) {
  if (!net_ok(net) || !g || n_outputs(net) != 4) return NAN;
  double* v0 = (double*)malloc(sizeof(double) * (size_t)orc_input_width(net));
  orc_features(net, p, t, v0, NULL);
  double y[4];
  mlp_outputs(net, v0, NULL, NULL, y);
  free(v0);
  for (int a = 0; a < 3; ++a) g[a] = y[1 + a];
  return sigmoid(y[0]);
}

int orc_eval_points(const orc_net* net, const double* xyz, int64_t n, double t, double* out) {
  if (!net_ok(net) || n < 0 || (n > 0 && (!xyz || !out))) return -1;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) out[i] = orc_density(net, xyz + 3 * i, t);
  return 0;
}

int orc_grad_points(const orc_net* net, const double* xyz, int64_t n, double t, double* out_d,
                    double* out_g) {
  if (!net_ok(net) || n < 0 || (n > 0 && (!xyz || !out_g))) return -1;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    double d = orc_density_grad_fwd(net, xyz + 3 * i, t, out_g + 3 * i);
    if (out_d) out_d[i] = d;
  }
  return 0;
}

/* -------------------------------------------------------- dense grids */

double orc_dense_sample(const double* vol, int nx, int ny, int nz, const double p[3]) {
  int i[3], n[3] = {nx, ny, nz};
  double f[3], df;
  for (int a = 0; a < 3; ++a) axis_cell(p[a], n[a], &i[a], &f[a], &df);
  double s = 0.0;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        double w = (cx ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) * (cz ? f[2] : 1.0 - f[2]);
        s += w * vol[((int64_t)(i[2] + cz) * ny + (i[1] + cy)) * nx + (i[0] + cx)];
      }
  return s;
}

int orc_dense_eval_points(const double* vol, int nx, int ny, int nz, const double* xyz,
                          int64_t n, double* out) {
  if (!vol || nx < 2 || ny < 2 || nz < 2 || n < 0 || (n > 0 && (!xyz || !out))) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = orc_dense_sample(vol, nx, ny, nz, xyz + 3 * i);
  return 0;
}

/* Marschner and Lobb's test signal on [-1,1]^3 with its analytic gradient:
   rho = (1 - sin(pi z / 2) + alpha (1 + cos(2 pi fm cos(pi r / 2)))) / (2 (1 + alpha)),
   r = sqrt(x^2 + y^2). */
double orc_marschner_lobb(double fm, double alpha, const double p[3], double g[3]) {
  const double x = p[0], y = p[1], z = p[2];
  const double r = sqrt(x * x + y * y);
  const double phi = 2.0 * M_PI * fm * cos(M_PI * r / 2.0);
  const double norm = 2.0 * (1.0 + alpha);
  if (g) {
    const double s_over_r = r > 1e-300 ? sin(M_PI * r / 2.0) / r : M_PI / 2.0;
    const double dr_common = alpha * sin(phi) * M_PI * M_PI * fm * s_over_r / norm;
    g[0] = dr_common * x;
    g[1] = dr_common * y;
    g[2] = -(M_PI / 2.0) * cos(M_PI * z / 2.0) / norm;
  }
  return (1.0 - sin(M_PI * z / 2.0) + alpha * (1.0 + cos(phi))) / norm;
}

double orc_field_density(const orc_field* f, const double p[3], double t, double g[3]) {
  switch (f->kind) {
    case ORC_FIELD_NET:
      if (g) return orc_density_grad_fwd(f->net, p, t, g);
      return orc_density(f->net, p, t);
    case ORC_FIELD_DENSE: {
      double d = orc_dense_sample(f->vol, f->nx, f->ny, f->nz, p);
      if (g) {
        /* central differences with a one-voxel step (Sec. 6) */
        const int n[3] = {f->nx, f->ny, f->nz};
        for (int a = 0; a < 3; ++a) {
          double h = 2.0 / (double)(n[a] - 1);
          double pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
          pp[a] += h;
          pm[a] -= h;
          g[a] = (orc_dense_sample(f->vol, f->nx, f->ny, f->nz, pp) -
                  orc_dense_sample(f->vol, f->nx, f->ny, f->nz, pm)) /
                 (2.0 * h);
        }
      }
      return d;
    }
    case ORC_FIELD_MARSCHNER_LOBB:
      return orc_marschner_lobb(f->ml_fm, f->ml_alpha, p, g);
    default:
      return NAN;
  }
}

/* -------------------------------------------- transfer function, camera */

/* Piecewise-linear TF (Sec. 3: density is mapped to colour and opacity);
   constant outside the first and last control points. */
int orc_tf_eval(const orc_tf* tf, double d, double rgba[4]) {
  if (!tf || tf->n < 2 || tf->n > 16) return -1;
  const int n = tf->n;
  if (!(d > tf->density[0])) {
    for (int q = 0; q < 4; ++q) rgba[q] = tf->rgba[0][q];
    return 0;
  }
  if (d >= tf->density[n - 1]) {
    for (int q = 0; q < 4; ++q) rgba[q] = tf->rgba[n - 1][q];
    return 0;
  }
  int j = 0;
  while (d >= tf->density[j + 1]) ++j;
  double w = (d - tf->density[j]) / (tf->density[j + 1] - tf->density[j]);
  for (int q = 0; q < 4; ++q) rgba[q] = (1.0 - w) * tf->rgba[j][q] + w * tf->rgba[j + 1][q];
  return 0;
}

static void normalize3(double v[3]) {
  double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= l;
  v[1] /= l;
  v[2] /= l;
}

static void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Look-at camera: forward f = target - eye, right = f x up, true up =
   right x f. Pixel centres at NDC ((2x+1)/W - 1, 1 - (2y+1)/H). */
int orc_camera_ray(const orc_camera* cam, int px, int py, double o[3], double dir[3]) {
  double f[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1],
                 cam->target[2] - cam->eye[2]};
  normalize3(f);
  double r[3], u[3];
  cross3(f, cam->up, r);
  normalize3(r);
  cross3(r, f, u);
  const double aspect = (double)cam->width / (double)cam->height;
  const double nx = (2.0 * px + 1.0) / cam->width - 1.0;
  const double ny = 1.0 - (2.0 * py + 1.0) / cam->height;
  if (cam->ortho) {
    const double h = cam->ortho_half_extent;
    for (int a = 0; a < 3; ++a) {
      o[a] = cam->eye[a] + h * (aspect * nx * r[a] + ny * u[a]);
      dir[a] = f[a];
    }
  } else {
    const double tn = tan(cam->fov_y_deg * M_PI / 360.0);
    for (int a = 0; a < 3; ++a) {
      o[a] = cam->eye[a];
      dir[a] = f[a] + tn * (aspect * nx * r[a] + ny * u[a]);
    }
    normalize3(dir);
  }
  return 0;
}

int orc_box_clip(const double o[3], const double dir[3], double* t0, double* t1) {
  double tn = -INFINITY, tf = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (dir[a] == 0.0) {
      if (o[a] < -1.0 || o[a] > 1.0) return 0;
      continue;
    }
    double ta = (-1.0 - o[a]) / dir[a], tb = (1.0 - o[a]) / dir[a];
    if (ta > tb) { double s = ta; ta = tb; tb = s; }
    if (ta > tn) tn = ta;
    if (tb < tf) tf = tb;
  }
  if (tn < 0.0) tn = 0.0;
  *t0 = tn;
  *t1 = tf;
  return tf > tn;
}

/* ------------------------------------------------------------ rendering */

/* Emission-absorption ray marching, front to back (Sec. 3, Sec. 5): the ray
   segment inside the box is cut into segments (fixed count, or a fixed step
   with the last segment clipped), each sampled at its midpoint. Per segment
   of length ds with extinction kappa = opacity_scale * alpha:
   a = 1 - exp(-kappa ds); C += T a rgb; A += T a; T *= exp(-kappa ds).
   The march stops after a sample once T < ert_eps. */
static void render_pixel(const orc_field* field, const orc_tf* tf, const orc_camera* cam,
                         const orc_march* m, int px, int py, double out[4], int64_t* samples) {
  double o[3], dir[3], t0, t1;
  out[0] = out[1] = out[2] = out[3] = 0.0;
  *samples = 0;
  orc_camera_ray(cam, px, py, o, dir);
  if (!orc_box_clip(o, dir, &t0, &t1)) return;
  int64_t nseg;
  double ds;
  if (m->fixed_steps > 0) {
    nseg = m->fixed_steps;
    ds = (t1 - t0) / (double)nseg;
  } else {
    ds = m->step;
    nseg = (int64_t)ceil((t1 - t0) / ds);
  }
  double T = 1.0, C[3] = {0.0, 0.0, 0.0}, A = 0.0;
  for (int64_t i = 0; i < nseg; ++i) {
    double a0 = t0 + (double)i * ds;
    double a1 = t0 + (double)(i + 1) * ds;
    if (m->fixed_steps <= 0 && a1 > t1) a1 = t1;
    double len = a1 - a0;
    if (len <= 0.0) break;
    double tm = 0.5 * (a0 + a1);
    double p[3] = {o[0] + tm * dir[0], o[1] + tm * dir[1], o[2] + tm * dir[2]};
    double g[3];
    double d;
    if (m->phong && m->grad_fd == 3 && field->kind == ORC_FIELD_NET) {
      /* backpropagation through the network to the position (the adjoint
         strategy of Sec. 6) */
      d = orc_density_grad_rev(field->net, p, cam->time, g);
    } else if (m->phong && m->grad_fd == 2 && field->kind == ORC_FIELD_NET) {
      /* the network's own gradient outputs (Sec. 6) */
      d = orc_density_grad_pred(field->net, p, cam->time, g);
    } else if (m->phong && m->grad_fd == 1 && field->kind == ORC_FIELD_NET) {
      /* finite differences of the network density: the centre and six
         central-difference samples, seven evaluations (Sec. 6) */
      d = orc_density(field->net, p, cam->time);
      for (int a = 0; a < 3; ++a) {
        double pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
        pp[a] += m->fd_step;
        pm[a] -= m->fd_step;
        g[a] = (orc_density(field->net, pp, cam->time) - orc_density(field->net, pm, cam->time)) /
               (2.0 * m->fd_step);
      }
    } else {
      d = orc_field_density(field, p, cam->time, m->phong ? g : NULL);
    }
    double rgba[4];
    orc_tf_eval(tf, d, rgba);
    if (m->phong) {
      /* Blinn-Phong with a headlight (light and view along -dir), normal =
         normalized density gradient (Sec. 6). */
      double gl = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
      if (gl >= 1e-6) {
        double ndl = fabs(-(g[0] * dir[0] + g[1] * dir[1] + g[2] * dir[2]) / gl);
        double spec = m->ks * pow(ndl, m->shininess);
        for (int q = 0; q < 3; ++q) rgba[q] = rgba[q] * (m->ka + m->kd * ndl) + spec;
      }
    }
    double kappa = tf->opacity_scale * rgba[3];
    double tr = exp(-kappa * len);
    double a = 1.0 - tr;
    for (int q = 0; q < 3; ++q) C[q] += T * a * rgba[q];
    A += T * a;
    T *= tr;
    ++*samples;
    if (T < m->ert_eps) break;
  }
  out[0] = C[0];
  out[1] = C[1];
  out[2] = C[2];
  out[3] = A;
}

int orc_render(const orc_field* field, const orc_tf* tf, const orc_camera* cams, int n_views,
               const orc_march* m, double* out, const int64_t* pixels, int64_t n_pix,
               int64_t* samples, int threads) {
  if (!field || !tf || !cams || !m || !out || n_views <= 0) return -1;
  if (tf->n < 2 || tf->n > 16) return -1;
  if (field->kind == ORC_FIELD_NET && !net_ok(field->net)) return -1;
  if (m->fixed_steps <= 0 && !(m->step > 0.0)) return -1;
  const int W = cams[0].width, Hh = cams[0].height;
  for (int v = 0; v < n_views; ++v)
    if (cams[v].width != W || cams[v].height != Hh || W <= 0 || Hh <= 0) return -1;
  const int64_t total = (int64_t)n_views * W * Hh;
  const int64_t count = pixels ? n_pix : total;
  int64_t nsamp = 0;
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nsamp) num_threads(threads)
#endif
  for (int64_t q = 0; q < count; ++q) {
    int64_t idx = pixels ? pixels[q] : q;
    if (idx < 0 || idx >= total) continue;
    int v = (int)(idx / ((int64_t)W * Hh));
    int64_t rem = idx % ((int64_t)W * Hh);
    int py = (int)(rem / W), px = (int)(rem % W);
    int64_t s;
    render_pixel(field, tf, &cams[v], m, px, py, out + 4 * idx, &s);
    nsamp += s;
  }
  if (samples) *samples = nsamp;
  return 0;
}

/* ------------------------------------------------------------- training */

/* World-space fitting (Sec. 3, Sec. 5): one forward pass per point keeping
   the layer inputs and pre-activations, then the chain rule backwards through
   the sigmoid, the layers (W_i^T) and the trilinear latent interpolation. */
int orc_train_grads(const orc_net* net, const double* xyz, const double* times, int64_t n,
                    const double* target, const double* target_grad, double grad_weight,
                    const double* dloss_dd, double* d_latent, double* d_weights, double* loss) {
  if (!net_ok(net) || n < 0 || !d_latent || !d_weights) return -1;
  if (n > 0 && (!xyz || (!target && !dloss_dd))) return -1;
  const int c = net->c, H = net->H, F = net->F, R = net->R, K0 = orc_input_width(net);
  const int64_t nw = orc_num_weights(net);
  const int64_t ng = (int64_t)net->K * R * R * R * F;
  memset(d_weights, 0, sizeof(double) * (size_t)nw);
  memset(d_latent, 0, sizeof(double) * (size_t)ng);
  const int mx = K0 > c ? K0 : c;
  /* per point: layer inputs h_0..h_H (h_0 = v0) and pre-activations */
  double* hs = (double*)malloc(sizeof(double) * ((size_t)K0 + (size_t)H * c + (size_t)H * c + 2 * (size_t)mx));
  double* pre = hs + K0 + (size_t)H * c;
  double* delta = pre + (size_t)H * c;
  double* dnext = delta + mx;
  double total = 0.0;
  for (int64_t q = 0; q < n; ++q) {
    const double* p = xyz + 3 * q;
    const double t = times ? times[q] : 0.0;
    orc_features(net, p, t, hs, NULL);
    /* forward */
    int width = K0;
    double* hin = hs;
    for (int i = 0; i < H; ++i) {
      const double* W = net->weights + layer_offset(net, i);
      const double* b = W + (int64_t)c * width;
      double* hout = hs + K0 + (size_t)i * c;
      for (int j = 0; j < c; ++j) {
        double s = b[j];
        for (int k = 0; k < width; ++k) s += W[(int64_t)j * width + k] * hin[k];
        pre[i * c + j] = s;
        hout[j] = act_f(net->act, s);
      }
      hin = hout;
      width = c;
    }
    const int no = n_outputs(net);
    const double* Wout = net->weights + layer_offset(net, H);
    double yo[4];
    for (int j = 0; j < no; ++j) {
      yo[j] = Wout[(int64_t)no * c + j];
      for (int k = 0; k < c; ++k) yo[j] += Wout[(int64_t)j * c + k] * hin[k];
    }
    double d = sigmoid(yo[0]);
    /* upstream dL/d output: the density through its sigmoid; the predicted
       gradient outputs (4-output networks with gradient targets) directly */
    double dy[4] = {0.0, 0.0, 0.0, 0.0};
    if (target) {
      double r = d - target[q];
      total += fabs(r);
      dy[0] = (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0)) / (double)n * d * (1.0 - d);
      if (no == 4 && target_grad)
        for (int a = 0; a < 3; ++a) {
          const double rg = yo[1 + a] - target_grad[3 * q + a];
          total += grad_weight / 3.0 * fabs(rg);
          dy[1 + a] = grad_weight / 3.0 * (rg > 0.0 ? 1.0 : (rg < 0.0 ? -1.0 : 0.0)) / (double)n;
        }
    } else {
      total += dloss_dd[q] * d;
      dy[0] = dloss_dd[q] * d * (1.0 - d);
    }
    /* output layer */
    double* dWout = d_weights + layer_offset(net, H);
    for (int k = 0; k < c; ++k) delta[k] = 0.0;
    for (int j = 0; j < no; ++j) {
      for (int k = 0; k < c; ++k) {
        dWout[(int64_t)j * c + k] += dy[j] * hin[k];
        delta[k] += dy[j] * Wout[(int64_t)j * c + k];
      }
      dWout[(int64_t)no * c + j] += dy[j];
    }
    /* activated layers, last to first */
    for (int i = H - 1; i >= 0; --i) {
      const int win = layer_in(net, i);
      const double* W = net->weights + layer_offset(net, i);
      double* dW = d_weights + layer_offset(net, i);
      double* db = dW + (int64_t)c * win;
      const double* x_in = i == 0 ? hs : hs + K0 + (size_t)(i - 1) * c;
      for (int j = 0; j < c; ++j) {
        delta[j] *= act_df(net->act, pre[i * c + j]);
        db[j] += delta[j];
        for (int k = 0; k < win; ++k) dW[(int64_t)j * win + k] += delta[j] * x_in[k];
      }
      for (int k = 0; k < win; ++k) {
        double s = 0.0;
        for (int j = 0; j < c; ++j) s += W[(int64_t)j * win + k] * delta[j];
        dnext[k] = s;
      }
      memcpy(delta, dnext, sizeof(double) * (size_t)win);
    }
    /* latent: delta[3..3+F) = dL/dz; scatter with the trilinear weights into
       the two keyframes the point's time interpolates (Sec. 8), each scaled by
       its blend weight (one keyframe, weight 1, when K == 1) */
    if (F > 0) {
      int ic[3];
      double fr[3], df;
      for (int a = 0; a < 3; ++a) axis_cell(p[a], R, &ic[a], &fr[a], &df);
      int key;
      double kw;
      key_pair(net, t, &key, &kw);
      const int nkeys = net->K > 1 ? 2 : 1;
      for (int kk = 0; kk < nkeys; ++kk) {
        const double bw = net->K > 1 ? (kk ? kw : 1.0 - kw) : 1.0;
        double* gk = d_latent + (int64_t)(key + kk) * R * R * R * F;
        for (int cz = 0; cz < 2; ++cz)
          for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
              double w = (cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) *
                         (cz ? fr[2] : 1.0 - fr[2]);
              double* gd = gk + ((((int64_t)(ic[2] + cz) * R + (ic[1] + cy)) * R + (ic[0] + cx)) * F);
              for (int ch = 0; ch < F; ++ch) gd[ch] += bw * w * delta[3 + ch];
            }
      }
    }
  }
  free(hs);
  if (loss) *loss = target ? (n > 0 ? total / (double)n : 0.0) : total;
  return 0;
}

int orc_quantize_grid(const float* src, int64_t n, int32_t F, uint8_t* codes, float* dequant) {
  if (n < 1 || F < 1 || !src || !codes || !dequant) return -1;
  for (int ch = 0; ch < F; ++ch) {
    float lo = src[ch], hi = src[ch];
    for (int64_t i = 1; i < n; ++i) {
      const float x = src[i * F + ch];
      if (x < lo) lo = x;
      if (x > hi) hi = x;
    }
    const float scale = (hi - lo) / 255.0f;
    dequant[2 * ch] = lo;
    dequant[2 * ch + 1] = scale;
    for (int64_t i = 0; i < n; ++i) {
      float q = 0.0f;
      if (scale > 0.0f) {
        q = nearbyintf((src[i * F + ch] - lo) / scale); /* default rounding: half to even */
        if (q < 0.0f) q = 0.0f;
        if (q > 255.0f) q = 255.0f;
      }
      codes[i * F + ch] = (uint8_t)q;
    }
  }
  return 0;
}

double orc_ssim(const double* a, const double* b, int H, int W, double* map) {
  const int r = 5;
  if (!a || !b || H < 2 * r + 1 || W < 2 * r + 1) return -1.0;
  double g[2 * r + 1][2 * r + 1], gs = 0.0;
  for (int i = -r; i <= r; ++i)
    for (int j = -r; j <= r; ++j) {
      g[i + r][j + r] = exp(-(double)(i * i + j * j) / (2.0 * 1.5 * 1.5));
      gs += g[i + r][j + r];
    }
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  double total = 0.0;
  const int HO = H - 2 * r, WO = W - 2 * r;
  for (int y = 0; y < HO; ++y)
    for (int x = 0; x < WO; ++x) {
      double s = 0.0;
      for (int ch = 0; ch < 3; ++ch) {
        double mx = 0.0, my = 0.0, xx = 0.0, yy = 0.0, xy = 0.0;
        for (int i = 0; i <= 2 * r; ++i)
          for (int j = 0; j <= 2 * r; ++j) {
            const double w = g[i][j] / gs;
            const double va = a[((int64_t)(y + i) * W + (x + j)) * 4 + ch];
            const double vb = b[((int64_t)(y + i) * W + (x + j)) * 4 + ch];
            mx += w * va;
            my += w * vb;
            xx += w * va * va;
            yy += w * vb * vb;
            xy += w * va * vb;
          }
        const double sx = xx - mx * mx, sy = yy - my * my, sxy = xy - mx * my;
        s += ((2.0 * mx * my + C1) * (2.0 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2));
      }
      s /= 3.0;
      if (map) map[(int64_t)y * WO + x] = s;
      total += s;
    }
  return total / ((double)HO * WO);
}

/* Adam (Kingma and Ba) with bias correction, as used for training in Sec. 5:
   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
   p -= lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps). */
int orc_adam(double* param, const double* grad, double* m, double* v, int64_t n, double lr,
             double beta1, double beta2, double eps, int32_t t) {
  if (n < 0 || t < 1 || (n > 0 && (!param || !grad || !m || !v))) return -1;
  const double bc1 = 1.0 - pow(beta1, (double)t);
  const double bc2 = 1.0 - pow(beta2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
    param[i] -= lr / bc1 * m[i] / (sqrt(v[i]) / sqrt(bc2) + eps);
  }
  return 0;
}

/* --------------------------------------- adaptive resampling (Sec. 5.4) */

/* Position inside voxel (ix, iy, iz) of a G^3 grid over [-1,1]^3 from three
   32-bit random words, in FP32 as stated in the header. */
static void voxel_position(int32_t G, int64_t v, const uint32_t* r3, float* p) {
  const int64_t ix = v % G, iy = (v / G) % G, iz = v / ((int64_t)G * G);
  const int64_t idx[3] = {ix, iy, iz};
  const float step = 2.0f / (float)G;
  for (int a = 0; a < 3; ++a) {
    const float u = (float)(r3[a] >> 8) * 5.9604644775390625e-8f; /* 2^-24 */
    p[a] = fmaf((float)idx[a] + u, step, -1.0f);
  }
}

int orc_voxel_points(int32_t G, int32_t per_voxel, const uint32_t* r, float* xyz) {
  if (G < 1 || per_voxel < 1 || !r || !xyz) return -1;
  const int64_t n = (int64_t)G * G * G * per_voxel;
  for (int64_t j = 0; j < n; ++j) voxel_position(G, j / per_voxel, r + 3 * j, xyz + 3 * j);
  return 0;
}

int orc_error_grid(const orc_net* net, const double* vol, int nx, int ny, int nz, const float* xyz,
                   int64_t n_voxels, int32_t per_voxel, double t, double* E) {
  if (!net_ok(net) || !vol || !xyz || !E || n_voxels < 0 || per_voxel < 1) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n_voxels; ++v) {
    double s = 0.0;
    for (int j = 0; j < per_voxel; ++j) {
      const float* q = xyz + 3 * (v * per_voxel + j);
      const double p[3] = {q[0], q[1], q[2]};
      s += fabs(orc_density(net, p, t) - orc_dense_sample(vol, nx, ny, nz, p));
    }
    E[v] = s / (double)per_voxel;
  }
  return 0;
}

int orc_weighted_points(const float* E, int32_t G, int64_t n, const uint32_t* r, float* xyz) {
  if (!E || G < 1 || n < 0 || (n > 0 && (!r || !xyz))) return -1;
  const int64_t nv = (int64_t)G * G * G;
  /* weights: E where E >= 0, else 0 */
  float emax = 0.0f;
  for (int64_t v = 0; v < nv; ++v)
    if (E[v] >= 0.0f && E[v] > emax) emax = E[v];
  const float scale = emax > 0.0f ? 16777216.0f / emax : 0.0f;
  uint64_t* Q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nv);
  uint64_t total = 0;
  for (int64_t v = 0; v < nv; ++v) {
    if (E[v] >= 0.0f) total += (uint64_t)floorf(E[v] * scale);
    Q[v] = total;
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t v;
    if (total == 0) {
      /* no weight anywhere: every voxel equally likely */
      v = (int64_t)(((uint64_t)r[4 * i] * (uint64_t)nv) >> 32);
    } else {
      const uint64_t target = (uint64_t)(((unsigned __int128)r[4 * i] * total) >> 32);
      int64_t lo = 0, hi = nv - 1; /* first v with Q[v] > target */
      while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (Q[mid] > target) hi = mid; else lo = mid + 1;
      }
      v = lo;
    }
    voxel_position(G, v, r + 4 * i + 1, xyz + 3 * i);
  }
  free(Q);
  return 0;
}
