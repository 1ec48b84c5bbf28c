// C ABI of the fV-SRN hot path: argument validation, host-side precomputation
// (camera bases, transfer-function segments, keyframe blends) and dispatch to
// the gfx950 kernels. Nothing here allocates device memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "../../include/fvsrn.h"
#include "fvsrn_launch.h"

using namespace fvsrn_detail;

namespace {

thread_local char g_err[512] = "";

fvsrn_status fail(fvsrn_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int n_outputs(const fvsrn_net_desc& d) { return d.num_outputs == 0 ? 1 : d.num_outputs; }

int time_inputs(const fvsrn_net_desc& d) {
  static const int n[4] = {0, 1, 8, 9};
  return (d.time_encoding >= 0 && d.time_encoding < 4) ? n[d.time_encoding] : 0;
}

int64_t num_weights(const fvsrn_net_desc& d) {
  const int64_t K0 = 3 + d.grid_channels + 6 * (int64_t)d.num_freqs + time_inputs(d), c = d.hidden_width,
                no = n_outputs(d);
  return c * K0 + c + (int64_t)(d.hidden_layers - 1) * (c * c + c) + no * c + no;
}

fvsrn_status check_desc(const fvsrn_net_desc* d) {
  if (!d) return fail(FVSRN_ERR_INVALID_ARGUMENT, "desc is NULL");
  if (d->grid_res < 2 || d->grid_res > 512)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "grid_res %d outside [2, 512]", d->grid_res);
  if (d->grid_channels < 1 || d->num_freqs < 0 || d->hidden_width < 1 || d->hidden_layers < 1)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "non-positive network dimension");
  if (d->num_keyframes < 1 || d->num_keyframes > 64)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "num_keyframes %d outside [1, 64]", d->num_keyframes);
  if (d->grid_dtype != FVSRN_F32 && d->grid_dtype != FVSRN_F16 && d->grid_dtype != FVSRN_U8)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "grid_dtype must be FVSRN_F32, FVSRN_F16 or FVSRN_U8");
  if (d->precision < FVSRN_F32 || d->precision > FVSRN_BF16)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "precision %d unknown", d->precision);
  if (d->activation < FVSRN_ACT_SINE || d->activation > FVSRN_ACT_IDENTITY)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "activation %d unknown", d->activation);
  const bool fl = (d->grid_channels == 8 || d->grid_channels == 16) && (d->num_freqs == 4 || d->num_freqs == 8);
  if (!fl)
    return fail(FVSRN_ERR_UNSUPPORTED, "(F, L) = (%d, %d) not compiled; supported F in {8, 16}, L in {4, 8}",
                d->grid_channels, d->num_freqs);
  if (d->hidden_width != 32 && d->hidden_width != 48 && d->hidden_width != 64)
    return fail(FVSRN_ERR_UNSUPPORTED, "hidden_width %d not compiled; supported 32, 48, 64", d->hidden_width);
  if (d->hidden_layers > 8) return fail(FVSRN_ERR_UNSUPPORTED, "hidden_layers %d > 8", d->hidden_layers);
  if (d->num_outputs != 0 && d->num_outputs != 1 && d->num_outputs != 4)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "num_outputs %d: must be 1 or 4 (0 means 1)", d->num_outputs);
  if (d->time_encoding < FVSRN_TIME_LATENT_ONLY || d->time_encoding > FVSRN_TIME_BOTH)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "time_encoding %d unknown", d->time_encoding);
  if (d->time_encoding != FVSRN_TIME_LATENT_ONLY &&
      !(d->time_hi > d->time_lo && d->time_hi - d->time_lo < 3.0e38f && d->time_lo > -3.0e38f))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "time encodings need finite time_lo < time_hi");
  if (d->fourier_matrix) {
    for (int j = 0; j < 9 * d->num_freqs; ++j)
      if (!(fabsf(d->fourier_matrix[j]) < 1.0e6f))
        return fail(FVSRN_ERR_INVALID_ARGUMENT, "fourier_matrix entry %d not finite or above 1e6", j);
    if (d->time_encoding != FVSRN_TIME_LATENT_ONLY)
      return fail(FVSRN_ERR_UNSUPPORTED, "a Fourier matrix together with a time encoding is not compiled");
  }
  // the kernels address one keyframe grid with 32-bit byte offsets
  const long long grid_bytes = (long long)d->grid_res * d->grid_res * d->grid_res * d->grid_channels *
                               (d->grid_dtype == FVSRN_U8 ? 1 : (d->grid_dtype == FVSRN_F16 ? 2 : 4));
  if (grid_bytes >= (1LL << 31))
    return fail(FVSRN_ERR_UNSUPPORTED, "one keyframe's latent grid is %lld bytes; at most 2^31 - 1 supported",
                grid_bytes);
  return FVSRN_OK;
}

fvsrn_status check_params(const fvsrn_net_desc* d, const fvsrn_params* p) {
  if (!p) return fail(FVSRN_ERR_INVALID_ARGUMENT, "params is NULL");
  if (!p->latent || !p->weights) return fail(FVSRN_ERR_INVALID_ARGUMENT, "latent or weights is NULL");
  if (!aligned16(p->latent) || !aligned16(p->weights))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "latent and weights must be 16-byte aligned");
  if (d->grid_dtype == FVSRN_U8 && (!p->latent_dequant || ((uintptr_t)p->latent_dequant & 7u)))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "uint8 grids need an 8-byte aligned latent_dequant");
  if (d->num_keyframes > 1) {
    if (!p->key_times) return fail(FVSRN_ERR_INVALID_ARGUMENT, "key_times required when K > 1");
    for (int k = 1; k < d->num_keyframes; ++k)
      if (!(p->key_times[k] > p->key_times[k - 1]))
        return fail(FVSRN_ERR_INVALID_ARGUMENT, "key_times must be strictly ascending");
  }
  return FVSRN_OK;
}

NetDev make_net(const fvsrn_net_desc* d, const void* latent, const float* weights,
                const float* dequant = nullptr) {
  NetDev n;
  n.latent = latent;
  n.weights = weights;
  n.R = d->grid_res;
  n.F = d->grid_channels;
  n.K = d->num_keyframes;
  n.L = d->num_freqs;
  n.C = d->hidden_width;
  n.H = d->hidden_layers;
  n.act = d->activation;
  n.grid_f16 = d->grid_dtype == FVSRN_F16;
  n.key_stride = (long long)d->grid_res * d->grid_res * d->grid_res * d->grid_channels;
  n.grid_u8 = d->grid_dtype == FVSRN_U8;
  n.dequant = n.grid_u8 ? dequant : nullptr;
  n.NO = n_outputs(*d);
  n.time_enc = d->time_encoding;
  n.t_lo = d->time_lo;
  n.t_hi = d->time_hi;
  n.t_scale = d->time_encoding ? (float)(2.0 / ((double)d->time_hi - d->time_lo)) : 0.0f;
  n.tau = 0.0f;
  n.fmat = d->fourier_matrix != nullptr;
  for (int j = 0; j < kMaxFourierRows; ++j)
    for (int a = 0; a < 3; ++a)
      n.fm[j][a] = (n.fmat && j < 3 * d->num_freqs) ? (float)(d->fourier_matrix[3 * j + a] / (2.0 * M_PI)) : 0.0f;
  return n;
}

// tau of time t for a time-encoded network: [lo, hi] onto [-1, 1], clamped.
float time_tau(const fvsrn_net_desc* d, float t) {
  if (!d->time_encoding) return 0.0f;
  const double tc = t < d->time_lo ? d->time_lo : (t > d->time_hi ? d->time_hi : t);
  return (float)(2.0 * (tc - d->time_lo) / ((double)d->time_hi - d->time_lo) - 1.0);
}

// Keyframe pair and blend weight for time t (clamped to the keyframe range).
void key_blend(const fvsrn_net_desc* d, const fvsrn_params* p, float t, int* key, float* w) {
  *key = 0;
  *w = 0.0f;
  const int K = d->num_keyframes;
  if (K <= 1) return;
  const float* kt = p->key_times;
  if (t <= kt[0]) return;
  if (t >= kt[K - 1]) {
    *key = K - 2;
    *w = 1.0f;
    return;
  }
  int j = 0;
  while (j + 1 < K - 1 && kt[j + 1] <= t) ++j;
  *key = j;
  *w = (float)(((double)t - kt[j]) / ((double)kt[j + 1] - kt[j]));
}

fvsrn_status make_tf(const fvsrn_tf* tf, TFDev* out) {
  if (!tf) return fail(FVSRN_ERR_INVALID_ARGUMENT, "tf is NULL");
  if (tf->n < 2 || tf->n > 16) return fail(FVSRN_ERR_INVALID_ARGUMENT, "tf.n %d outside [2, 16]", tf->n);
  for (int j = 1; j < tf->n; ++j)
    if (!(tf->density[j] > tf->density[j - 1]))
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "tf densities must be strictly ascending");
  if (!(tf->opacity_scale >= 0.0f)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "tf.opacity_scale < 0");
  memset(out, 0, sizeof(*out));
  out->n_seg = tf->n - 1;
  const double s = tf->opacity_scale;
  for (int q = 0; q < 4; ++q) out->base[q] = (float)(tf->rgba[0][q] * (q == 3 ? s : 1.0));
  for (int j = 0; j + 1 < tf->n; ++j) {
    const double inv = 1.0 / ((double)tf->density[j + 1] - tf->density[j]);
    out->inv[j] = (float)inv;
    out->off[j] = (float)(-(double)tf->density[j] * inv);
    for (int q = 0; q < 4; ++q)
      out->delta[j][q] = (float)(((double)tf->rgba[j + 1][q] - tf->rgba[j][q]) * (q == 3 ? s : 1.0));
  }
  return FVSRN_OK;
}

fvsrn_status make_views(const fvsrn_camera* cams, int n_views, int first, int count,
                        const fvsrn_net_desc* d, const fvsrn_params* p, ViewBatch* vb) {
  memset(vb, 0, sizeof(*vb));
  vb->n_views = count;
  vb->width = cams[0].width;
  vb->height = cams[0].height;
  (void)n_views;
  for (int v = 0; v < count; ++v) {
    const fvsrn_camera& c = cams[first + v];
    CamDev& o = vb->cam[v];
    double f[3] = {(double)c.target[0] - c.eye[0], (double)c.target[1] - c.eye[1],
                   (double)c.target[2] - c.eye[2]};
    double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "camera %d: eye == target", first + v);
    for (int a = 0; a < 3; ++a) f[a] /= fl;
    double r[3] = {f[1] * c.up[2] - f[2] * c.up[1], f[2] * c.up[0] - f[0] * c.up[2],
                   f[0] * c.up[1] - f[1] * c.up[0]};
    double rl = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 0.0)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "camera %d: up parallel to view", first + v);
    for (int a = 0; a < 3; ++a) r[a] /= rl;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    for (int a = 0; a < 3; ++a) {
      o.eye[a] = c.eye[a];
      o.fwd[a] = f[a];
      o.right[a] = r[a];
      o.up[a] = u[a];
    }
    o.tan_half = tan((double)c.fov_y_deg * M_PI / 360.0);
    o.half_extent = c.ortho_half_extent;
    o.aspect = (double)c.width / (double)c.height;
    o.ortho = c.ortho ? 1 : 0;
    if (d && p) key_blend(d, p, c.time, &o.key, &o.key_w);
    o.tau = d ? time_tau(d, c.time) : 0.0f;
  }
  return FVSRN_OK;
}

fvsrn_status check_cams(const fvsrn_camera* cams, int32_t n_views, const fvsrn_march* m) {
  if (!cams || !m) return fail(FVSRN_ERR_INVALID_ARGUMENT, "cams or march is NULL");
  if (n_views <= 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n_views must be positive");
  for (int v = 0; v < n_views; ++v) {
    if (cams[v].width <= 0 || cams[v].height <= 0 || cams[v].width > 16384 || cams[v].height > 16384)
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "camera %d: image size out of range", v);
    if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "all cameras must share width and height");
    if (!cams[v].ortho && !(cams[v].fov_y_deg > 0.0f && cams[v].fov_y_deg < 180.0f))
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "camera %d: fov_y_deg outside (0, 180)", v);
  }
  if (m->fixed_steps < 0 || m->fixed_steps > (1 << 20))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "fixed_steps outside [0, 2^20]");
  // a ray crosses at most 2 sqrt(3) world units: this bounds a march to ~2.3e5 steps
  if (m->fixed_steps == 0 && !(m->step >= 1.0f / 65536.0f))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "step must be >= 2^-16 world units");
  if (!(m->ert_eps >= 0.0f) || m->ert_eps > 1.0f) return fail(FVSRN_ERR_INVALID_ARGUMENT, "ert_eps outside [0, 1]");
  if (m->grad_mode != FVSRN_GRAD_FORWARD && m->grad_mode != FVSRN_GRAD_CENTRAL &&
      m->grad_mode != FVSRN_GRAD_PREDICTED && m->grad_mode != FVSRN_GRAD_ADJOINT)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "grad_mode unknown");
  if (m->phong && m->grad_mode == FVSRN_GRAD_CENTRAL && !(m->fd_step > 0.0f && m->fd_step < 1.0f))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "fd_step must be in (0, 1) for central differences");
  // Phong coefficients: finite and non-negative (a negative shininess would
  // raise |n.l| = 0 to an infinite power)
  if (m->phong) {
    const float k[4] = {m->ka, m->kd, m->ks, m->shininess};
    static const char* names[4] = {"ka", "kd", "ks", "shininess"};
    for (int j = 0; j < 4; ++j)
      if (!(k[j] >= 0.0f && k[j] <= 1.0e6f))
        return fail(FVSRN_ERR_INVALID_ARGUMENT, "phong %s must be finite, >= 0 and <= 1e6", names[j]);
  }
  return FVSRN_OK;
}

MarchDev make_march(const fvsrn_march* m) {
  MarchDev o;
  o.step = m->step;
  o.fixed_steps = m->fixed_steps;
  o.ert_eps = m->ert_eps;
  o.phong = m->phong ? 1 : 0;
  o.ka = m->ka;
  o.kd = m->kd;
  o.ks = m->ks;
  o.shininess = m->shininess;
  o.grad_mode = m->grad_mode;
  o.fd_step = m->fd_step;
  return o;
}

fvsrn_status launch_status(int rc, const char* what) {
  if (rc == 0) return FVSRN_OK;
  if (rc == 1) return fail(FVSRN_ERR_UNSUPPORTED, "%s: configuration not compiled", what);
  if (rc == kLaunchNoLds)
    return fail(FVSRN_ERR_UNSUPPORTED, "%s: the network's weight fragments do not fit the 160 KiB of LDS", what);
  if (rc == kLaunchTooLarge) return fail(FVSRN_ERR_UNSUPPORTED, "%s: launch exceeds a 32-bit grid", what);
  return fail(FVSRN_ERR_DEVICE, "%s: launch failed: %s", what, last_hip_error());
}

}  // namespace

extern "C" {

int64_t fvsrn_num_weights(const fvsrn_net_desc* desc) {
  if (!desc || desc->hidden_layers < 1 || desc->hidden_width < 1 || desc->grid_channels < 0 ||
      desc->num_freqs < 0)
    return 0;
  return num_weights(*desc);
}

const char* fvsrn_status_str(fvsrn_status s) {
  switch (s) {
    case FVSRN_OK: return "ok";
    case FVSRN_ERR_INVALID_ARGUMENT: return "invalid argument";
    case FVSRN_ERR_UNSUPPORTED: return "unsupported configuration";
    case FVSRN_ERR_WORKSPACE: return "workspace too small";
    case FVSRN_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* fvsrn_last_error(void) { return g_err; }

#ifndef FVSRN_SOURCE_HASH
#error "FVSRN_SOURCE_HASH must be defined by the build (hash of the sources)"
#endif
const char* fvsrn_build_id(void) { return FVSRN_SOURCE_HASH; }

fvsrn_status fvsrn_render(const fvsrn_net_desc* desc, const fvsrn_params* params, const fvsrn_tf* tf,
                          const fvsrn_camera* cams, int32_t n_views, const fvsrn_march* march,
                          float* out_rgba, unsigned long long* stats, void* stream) {
  g_err[0] = 0;
  fvsrn_status s;
  if ((s = check_desc(desc)) != FVSRN_OK) return s;
  if ((s = check_params(desc, params)) != FVSRN_OK) return s;
  if ((s = check_cams(cams, n_views, march)) != FVSRN_OK) return s;
  if (march->phong && march->grad_mode == FVSRN_GRAD_PREDICTED && n_outputs(*desc) != 4)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "predicted gradients need a network with num_outputs == 4");
  if (!out_rgba || !aligned16(out_rgba)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "out_rgba NULL or misaligned");
  if (stats && ((uintptr_t)stats & 7u)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "stats misaligned");
  TFDev tfd;
  if ((s = make_tf(tf, &tfd)) != FVSRN_OK) return s;
  const NetDev nd = make_net(desc, params->latent, params->weights, params->latent_dequant);
  const MarchDev md = make_march(march);
  const long long per_view = (long long)cams[0].width * cams[0].height * 4;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsPerLaunch) {
    const int cnt = n_views - v0 < kMaxViewsPerLaunch ? n_views - v0 : kMaxViewsPerLaunch;
    ViewBatch vb;
    if ((s = make_views(cams, n_views, v0, cnt, desc, params, &vb)) != FVSRN_OK) return s;
    const int rc = launch_render(nd, desc->precision, tfd, vb, md, out_rgba + v0 * per_view, stats, stream);
    if ((s = launch_status(rc, "fvsrn_render")) != FVSRN_OK) return s;
  }
  return FVSRN_OK;
}

fvsrn_status fvsrn_eval_points(const fvsrn_net_desc* desc, const fvsrn_params* params, const float* xyz,
                               int64_t n, float time, float* out_density, void* stream) {
  g_err[0] = 0;
  if (n > 0 && !out_density) return fail(FVSRN_ERR_INVALID_ARGUMENT, "out_density is NULL");
  fvsrn_status s;
  if ((s = check_desc(desc)) != FVSRN_OK) return s;
  if ((s = check_params(desc, params)) != FVSRN_OK) return s;
  if (n < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n < 0");
  if (n == 0) return FVSRN_OK;
  if (!xyz || !aligned16(xyz) || !aligned16(out_density))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz / out_density NULL or misaligned");
  int key;
  float kw;
  key_blend(desc, params, time, &key, &kw);
  NetDev nd = make_net(desc, params->latent, params->weights, params->latent_dequant);
  nd.tau = time_tau(desc, time);
  return launch_status(launch_points(nd, desc->precision, xyz, n, key, kw, out_density, nullptr, 0, stream),
                       "fvsrn_eval_points");
}

fvsrn_status fvsrn_grad_points(const fvsrn_net_desc* desc, const fvsrn_params* params, const float* xyz,
                               int64_t n, float time, int32_t grad_mode, float* out_density, float* out_grad,
                               void* stream) {
  g_err[0] = 0;
  if (n > 0 && !out_grad) return fail(FVSRN_ERR_INVALID_ARGUMENT, "out_grad is NULL");
  fvsrn_status s;
  if ((s = check_desc(desc)) != FVSRN_OK) return s;
  if ((s = check_params(desc, params)) != FVSRN_OK) return s;
  if (grad_mode != FVSRN_GRAD_FORWARD && grad_mode != FVSRN_GRAD_ADJOINT && grad_mode != FVSRN_GRAD_PREDICTED)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "grad_mode must be FORWARD, ADJOINT or PREDICTED for points");
  if (grad_mode == FVSRN_GRAD_PREDICTED && n_outputs(*desc) != 4)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "predicted gradients need a network with num_outputs == 4");
  if (n < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n < 0");
  if (n == 0) return FVSRN_OK;
  if (!xyz || !aligned16(xyz) || !aligned16(out_grad) || (out_density && !aligned16(out_density)))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz / outputs NULL or misaligned");
  int key;
  float kw;
  key_blend(desc, params, time, &key, &kw);
  NetDev nd = make_net(desc, params->latent, params->weights, params->latent_dequant);
  nd.tau = time_tau(desc, time);
  return launch_status(launch_points(nd, desc->precision, xyz, n, key, kw, out_density, out_grad, grad_mode, stream),
                       "fvsrn_grad_points");
}

size_t fvsrn_train_workspace_size(const fvsrn_net_desc* desc, int64_t n) {
  if (check_desc(desc) != FVSRN_OK || n < 0) return 0;
  const NetDev nd = make_net(desc, nullptr, nullptr);
  return train_workspace_bytes(nd, n);
}

}  // extern "C"

namespace {

// fvsrn_train_step with the caller's workspace, or (static_ws) with the
// library's per-GPU static workspace.
fvsrn_status train_step_impl(const fvsrn_net_desc* desc, float* latent, float* weights, const float* key_times,
                             float* d_latent, float* d_weights, const float* xyz, const float* times, int64_t n,
                             const float* target, const float* target_grad, float grad_weight,
                             const float* dloss_dy, const fvsrn_adam* adam, float* out_loss, void* workspace,
                             size_t workspace_bytes, bool static_ws, void* stream) {
  g_err[0] = 0;
  fvsrn_status s;
  if ((s = check_desc(desc)) != FVSRN_OK) return s;
  const fvsrn_params kp = {latent, weights, key_times, nullptr};
  if ((s = check_params(desc, &kp)) != FVSRN_OK) return s;
  if (n > 0 && times && ((uintptr_t)times & 3u)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "times misaligned");
  // a point's keyframe pair is selected per lane: the K grids are addressed
  // with 32-bit byte offsets from the first one
  const long long all_bytes = (long long)desc->num_keyframes * desc->grid_res * desc->grid_res * desc->grid_res *
                              desc->grid_channels * 4;
  if (all_bytes >= (1LL << 31)) return fail(FVSRN_ERR_UNSUPPORTED, "training: K latent grids above 2^31 bytes");
  if (desc->grid_dtype != FVSRN_F32) return fail(FVSRN_ERR_UNSUPPORTED, "training needs an FP32 latent grid");
  if (desc->precision != FVSRN_F32 && desc->precision != FVSRN_F16)
    return fail(FVSRN_ERR_UNSUPPORTED, "training runs in FP32 or FP16");
  if (desc->precision == FVSRN_F16 &&
      (dloss_dy || desc->time_encoding != FVSRN_TIME_LATENT_ONLY || desc->fourier_matrix))
    return fail(FVSRN_ERR_UNSUPPORTED,
                "FP16 training: L1 targets only, without time inputs or a Fourier matrix (use FP32)");
  if (!latent || !weights || !d_latent || !d_weights)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "latent, weights, d_latent, d_weights must be non-NULL");
  if (!aligned16(latent) || !aligned16(weights) || !aligned16(d_latent) || !aligned16(d_weights))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "parameter buffers must be 16-byte aligned");
  if (n < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n < 0");
  if (n > 0 && (!xyz || !aligned16(xyz))) return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz NULL or misaligned");
  if (n > 0 && !target && !dloss_dy) return fail(FVSRN_ERR_INVALID_ARGUMENT, "target or dloss_dy required");
  if (target_grad) {
    if (!target) return fail(FVSRN_ERR_INVALID_ARGUMENT, "target_grad needs target (L1 mode)");
    if (n_outputs(*desc) != 4)
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "target_grad needs a network with num_outputs == 4");
    if (!(grad_weight >= 0.0f) || grad_weight > 1e30f)
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "grad_weight must be finite and >= 0");
    if ((uintptr_t)target_grad & 3u) return fail(FVSRN_ERR_INVALID_ARGUMENT, "target_grad misaligned");
  }
  if (adam) {
    if (adam->step < 1) return fail(FVSRN_ERR_INVALID_ARGUMENT, "adam.step must be >= 1");
    if (!adam->m_latent || !adam->v_latent || !adam->m_weights || !adam->v_weights)
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "adam moment buffers must be non-NULL");
  }
  const NetDev nd = make_net(desc, latent, weights);
  if (n >= (1LL << 31)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "training takes fewer than 2^31 points per step");
  const size_t need = train_workspace_bytes(nd, n);
  if (static_ws) {
    if (need > kStaticTrainScratchBytes)
      return fail(FVSRN_ERR_WORKSPACE,
                  "fvsrn_train_step_noalloc: this step needs %zu bytes of workspace, above the static %zu; "
                  "use fvsrn_train_step or fewer points",
                  need, kStaticTrainScratchBytes);
    if (static_train_scratch(&workspace) != 0)
      return fail(FVSRN_ERR_DEVICE, "fvsrn_train_step_noalloc: static workspace address lookup failed");
    workspace_bytes = kStaticTrainScratchBytes;
  } else if (need > 0 && (!workspace || ((uintptr_t)workspace & 15u) || workspace_bytes < need)) {
    return fail(FVSRN_ERR_WORKSPACE, "workspace of %zu bytes (16-byte aligned) required", need);
  }
  KeyTimes kt;
  kt.K = desc->num_keyframes;
  for (int k = 0; k < kMaxKeyframes; ++k) kt.t[k] = (k < kt.K && key_times) ? key_times[k] : 0.0f;
  const int rc = launch_train(nd, kt, latent, weights, d_latent, d_weights, xyz, times, n, target, target_grad,
                              target_grad ? grad_weight : 0.0f, dloss_dy, adam != nullptr,
                              adam ? adam->lr_grid : 0.f, adam ? adam->lr_mlp : 0.f, adam ? adam->beta1 : 0.f,
                              adam ? adam->beta2 : 0.f, adam ? adam->eps : 0.f, adam ? adam->step : 0,
                              adam ? adam->m_latent : nullptr, adam ? adam->v_latent : nullptr,
                              adam ? adam->m_weights : nullptr, adam ? adam->v_weights : nullptr, out_loss,
                              workspace, workspace_bytes, desc->precision == FVSRN_F16 ? 1 : 0, stream);
  return launch_status(rc, static_ws ? "fvsrn_train_step_noalloc" : "fvsrn_train_step");
}

}  // namespace

extern "C" {

fvsrn_status fvsrn_train_step(const fvsrn_net_desc* desc, float* latent, float* weights, const float* key_times,
                              float* d_latent, float* d_weights, const float* xyz, const float* times, int64_t n,
                              const float* target, const float* target_grad, float grad_weight,
                              const float* dloss_dy, const fvsrn_adam* adam, float* out_loss,
                              void* workspace, size_t workspace_bytes, void* stream) {
  return train_step_impl(desc, latent, weights, key_times, d_latent, d_weights, xyz, times, n, target, target_grad,
                         grad_weight, dloss_dy, adam, out_loss, workspace, workspace_bytes, false, stream);
}

fvsrn_status fvsrn_train_step_noalloc(const fvsrn_net_desc* desc, float* latent, float* weights,
                                      const float* key_times, float* d_latent, float* d_weights, const float* xyz,
                                      const float* times, int64_t n, const float* target, const float* target_grad,
                                      float grad_weight, const float* dloss_dy, const fvsrn_adam* adam,
                                      float* out_loss, void* stream) {
  return train_step_impl(desc, latent, weights, key_times, d_latent, d_weights, xyz, times, n, target, target_grad,
                         grad_weight, dloss_dy, adam, out_loss, nullptr, 0, true, stream);
}

fvsrn_status fvsrn_ssim_map(const float* a, const float* b, int32_t width, int32_t height, int32_t n_images,
                            float* out_map, void* stream) {
  g_err[0] = 0;
  if (width < 11 || height < 11) return fail(FVSRN_ERR_INVALID_ARGUMENT, "images need at least 11 x 11 pixels");
  if (n_images < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n_images < 0");
  if (n_images == 0) return FVSRN_OK;
  if (!a || !b || !out_map || !aligned16(a) || !aligned16(b) || ((uintptr_t)out_map & 3u))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "a, b, out_map NULL or misaligned");
  return launch_status(launch_ssim(a, b, width, height, n_images, out_map, stream), "fvsrn_ssim_map");
}

fvsrn_status fvsrn_quantize_grid(const float* src, int64_t n_vertices, int32_t channels, uint8_t* codes,
                                 float* dequant, void* stream) {
  g_err[0] = 0;
  if (n_vertices < 1) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n_vertices < 1");
  if (channels < 1 || channels > 64) return fail(FVSRN_ERR_INVALID_ARGUMENT, "channels outside [1, 64]");
  if (!src || !codes || !dequant || ((uintptr_t)src & 3u) || ((uintptr_t)dequant & 7u))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "src, codes, dequant NULL or misaligned");
  return launch_status(launch_quantize(src, n_vertices, channels, codes, dequant, stream), "fvsrn_quantize_grid");
}

fvsrn_status fvsrn_render_dense(const float* vol, int32_t nx, int32_t ny, int32_t nz, const fvsrn_tf* tf,
                                const fvsrn_camera* cams, int32_t n_views, const fvsrn_march* march,
                                float* out_rgba, unsigned long long* stats, void* stream) {
  g_err[0] = 0;
  fvsrn_status s;
  if (!vol || !aligned16(vol)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "vol NULL or misaligned");
  if (nx < 2 || ny < 2 || nz < 2) return fail(FVSRN_ERR_INVALID_ARGUMENT, "volume needs >= 2 vertices per axis");
  if ((s = check_cams(cams, n_views, march)) != FVSRN_OK) return s;
  if (!out_rgba || !aligned16(out_rgba)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "out_rgba NULL or misaligned");
  if (stats && ((uintptr_t)stats & 7u)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "stats misaligned");
  TFDev tfd;
  if ((s = make_tf(tf, &tfd)) != FVSRN_OK) return s;
  const MarchDev md = make_march(march);
  const long long per_view = (long long)cams[0].width * cams[0].height * 4;
  for (int v0 = 0; v0 < n_views; v0 += kMaxViewsPerLaunch) {
    const int cnt = n_views - v0 < kMaxViewsPerLaunch ? n_views - v0 : kMaxViewsPerLaunch;
    ViewBatch vb;
    if ((s = make_views(cams, n_views, v0, cnt, nullptr, nullptr, &vb)) != FVSRN_OK) return s;
    const int rc = launch_render_dense(vol, nx, ny, nz, tfd, vb, md, out_rgba + v0 * per_view, stats, stream);
    if ((s = launch_status(rc, "fvsrn_render_dense")) != FVSRN_OK) return s;
  }
  return FVSRN_OK;
}

fvsrn_status fvsrn_dense_eval_points(const float* vol, int32_t nx, int32_t ny, int32_t nz, const float* xyz,
                                     int64_t n, float* out, void* stream) {
  g_err[0] = 0;
  if (!vol || !aligned16(vol)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "vol NULL or misaligned");
  if (nx < 2 || ny < 2 || nz < 2) return fail(FVSRN_ERR_INVALID_ARGUMENT, "volume needs >= 2 vertices per axis");
  if (n < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n < 0");
  if (n == 0) return FVSRN_OK;
  if (!xyz || !out || !aligned16(xyz) || !aligned16(out))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz / out NULL or misaligned");
  return launch_status(launch_dense_points(vol, nx, ny, nz, xyz, n, out, nullptr, stream),
                       "fvsrn_dense_eval_points");
}

fvsrn_status fvsrn_dense_grad_points(const float* vol, int32_t nx, int32_t ny, int32_t nz, const float* xyz,
                                     int64_t n, float* out_density, float* out_grad, void* stream) {
  g_err[0] = 0;
  if (!vol || !aligned16(vol)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "vol NULL or misaligned");
  if (nx < 2 || ny < 2 || nz < 2) return fail(FVSRN_ERR_INVALID_ARGUMENT, "volume needs >= 2 vertices per axis");
  if (n < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n < 0");
  if (n == 0) return FVSRN_OK;
  if (!xyz || !out_grad || !aligned16(xyz) || ((uintptr_t)out_grad & 3u) ||
      (out_density && ((uintptr_t)out_density & 3u)))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz / out_grad NULL or misaligned");
  return launch_status(launch_dense_points(vol, nx, ny, nz, xyz, n, out_density, out_grad, stream),
                       "fvsrn_dense_grad_points");
}

fvsrn_status fvsrn_sample_points(uint64_t seed, uint64_t counter, int64_t n, float* xyz, void* stream) {
  g_err[0] = 0;
  if (n < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n < 0");
  if (n == 0) return FVSRN_OK;
  if (!xyz || !aligned16(xyz)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz NULL or misaligned");
  return launch_status(launch_sample_points(seed, counter, n, xyz, stream), "fvsrn_sample_points");
}

fvsrn_status fvsrn_voxel_points(uint64_t seed, uint64_t counter, int32_t G, int32_t per_voxel, float* xyz,
                                void* stream) {
  g_err[0] = 0;
  if (G < 1 || per_voxel < 1) return fail(FVSRN_ERR_INVALID_ARGUMENT, "G and per_voxel must be >= 1");
  if ((long long)G * G * G * per_voxel >= (1LL << 32))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "G^3 * per_voxel must stay below 2^32");
  if (!xyz || !aligned16(xyz)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz NULL or misaligned");
  return launch_status(launch_voxel_points(seed, counter, G, per_voxel, xyz, stream), "fvsrn_voxel_points");
}

fvsrn_status fvsrn_error_grid(const fvsrn_net_desc* desc, const fvsrn_params* params, const float* vol, int32_t nx,
                              int32_t ny, int32_t nz, const float* xyz, int64_t n_voxels, int32_t per_voxel,
                              float time, float* E, float* scratch, void* stream) {
  g_err[0] = 0;
  fvsrn_status s;
  if ((s = check_desc(desc)) != FVSRN_OK) return s;
  if ((s = check_params(desc, params)) != FVSRN_OK) return s;
  if (desc->precision != FVSRN_F32) return fail(FVSRN_ERR_UNSUPPORTED, "the error grid uses an FP32 network");
  if (!vol || !aligned16(vol)) return fail(FVSRN_ERR_INVALID_ARGUMENT, "vol NULL or misaligned");
  if (nx < 2 || ny < 2 || nz < 2) return fail(FVSRN_ERR_INVALID_ARGUMENT, "volume needs >= 2 vertices per axis");
  if (n_voxels < 0 || per_voxel < 1) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n_voxels < 0 or per_voxel < 1");
  if (n_voxels == 0) return FVSRN_OK;
  if (!xyz || !E || !scratch || !aligned16(xyz) || !aligned16(scratch) || ((uintptr_t)E & 3u))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz, E, scratch NULL or misaligned");
  int key;
  float kw;
  key_blend(desc, params, time, &key, &kw);
  NetDev nd = make_net(desc, params->latent, params->weights, params->latent_dequant);
  nd.tau = time_tau(desc, time);
  const long long n = n_voxels * (long long)per_voxel;
  if ((s = launch_status(launch_points(nd, desc->precision, xyz, n, key, kw, scratch, nullptr, 0, stream),
                         "fvsrn_error_grid")) != FVSRN_OK)
    return s;
  return launch_status(launch_error_reduce(scratch, vol, nx, ny, nz, xyz, n_voxels, per_voxel, E, stream),
                       "fvsrn_error_grid");
}

size_t fvsrn_weighted_points_workspace_size(int32_t G) {
  if (G < 1 || G > 1024) return 0;
  return weighted_points_workspace_bytes((long long)G * G * G);
}

fvsrn_status fvsrn_sample_points_weighted(uint64_t seed, uint64_t counter, const float* E, int32_t G, int64_t n,
                                          float* xyz, void* workspace, size_t workspace_bytes, void* stream) {
  g_err[0] = 0;
  if (G < 1 || G > 1024) return fail(FVSRN_ERR_INVALID_ARGUMENT, "G outside [1, 1024]");
  if (n < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n < 0");
  if ((uintptr_t)E & 3u) return fail(FVSRN_ERR_INVALID_ARGUMENT, "E misaligned");
  if (n > 0 && (!xyz || !aligned16(xyz))) return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz NULL or misaligned");
  const size_t need = weighted_points_workspace_bytes((long long)G * G * G);
  if (!workspace || ((uintptr_t)workspace & 15u) || workspace_bytes < need)
    return fail(FVSRN_ERR_WORKSPACE, "workspace of %zu bytes (16-byte aligned) required", need);
  return launch_status(launch_weighted_points(seed, counter, E, G, n, xyz, workspace, stream),
                       "fvsrn_sample_points_weighted");
}

fvsrn_status fvsrn_sample_points_weighted_multi(uint64_t seed, uint64_t counter, int32_t G, int32_t n_grids,
                                                const int64_t* n_per_grid, float* xyz, const void* workspace,
                                                size_t workspace_stride, void* stream) {
  g_err[0] = 0;
  if (G < 1 || G > 1024) return fail(FVSRN_ERR_INVALID_ARGUMENT, "G outside [1, 1024]");
  if (n_grids < 1 || n_grids > kMaxDrawGrids)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "n_grids outside [1, %d]", kMaxDrawGrids);
  if (!n_per_grid) return fail(FVSRN_ERR_INVALID_ARGUMENT, "n_per_grid NULL");
  long long n = 0;
  for (int k = 0; k < n_grids; ++k) {
    if (n_per_grid[k] < 0 || n_per_grid[k] > (1LL << 40))
      return fail(FVSRN_ERR_INVALID_ARGUMENT, "n_per_grid[%d] outside [0, 2^40]", k);
    n += n_per_grid[k];
  }
  if (n > 0 && (!xyz || !aligned16(xyz))) return fail(FVSRN_ERR_INVALID_ARGUMENT, "xyz NULL or misaligned");
  const size_t need = weighted_points_workspace_bytes((long long)G * G * G);
  if (!workspace || ((uintptr_t)workspace & 15u) || (workspace_stride & 15u) || workspace_stride < need)
    return fail(FVSRN_ERR_WORKSPACE, "workspace slices of at least %zu bytes, 16-byte aligned, required", need);
  return launch_status(
      launch_weighted_points_multi(seed, counter, G, n_grids, n_per_grid, xyz, workspace, workspace_stride, stream),
      "fvsrn_sample_points_weighted_multi");
}

fvsrn_status fvsrn_cast_grid(const float* src, void* dst, int64_t count, int32_t dst_dtype, void* stream) {
  g_err[0] = 0;
  if (count < 0) return fail(FVSRN_ERR_INVALID_ARGUMENT, "count < 0");
  if (dst_dtype != FVSRN_F16 && dst_dtype != FVSRN_BF16)
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "dst_dtype must be FVSRN_F16 or FVSRN_BF16");
  if (count == 0) return FVSRN_OK;
  if (!src || !dst || !aligned16(src) || !aligned16(dst))
    return fail(FVSRN_ERR_INVALID_ARGUMENT, "src / dst NULL or misaligned");
  return launch_status(launch_cast(src, dst, count, dst_dtype, stream), "fvsrn_cast_grid");
}

}  // extern "C"
