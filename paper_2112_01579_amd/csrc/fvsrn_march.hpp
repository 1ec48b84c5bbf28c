// Fused fV-SRN ray-march and point-evaluation kernels, templated on the
// network configuration and shading mode; the per-precision units
// (fvsrn_march.hip, fvsrn_adjoint.hip) instantiate and dispatch them.
//
// Render: one wavefront owns a tile of rays -- 8x8 pixels without shading,
// 4x4 pixels (four lanes per ray: value and three tangents) for forward-mode
// gradients, 4x2 pixels (eight lanes per ray: centre and six central-difference
// neighbours) for finite-difference gradients; a network that predicts its own
// gradient (four outputs) and the adjoint (reverse-mode) gradient shade from
// 8x8 tiles like the unshaded render. Per march step every lane builds its
// input row, the wave runs the MLP on the matrix cores, and the ray-owning
// lanes map the density through the transfer function and composite front to
// back (Sec. 3, Sec. 4), stopping when the transmittance falls below the
// termination threshold.
#pragma once
#include "fvsrn_adjoint.hpp"

namespace fvsrn_detail {

namespace {

// Shading modes of the render kernel: none, forward-mode gradient, central
// differences, the network's predicted gradient, the adjoint (Sec. 6).
enum { kShadeNone = 0, kShadeFwd = 1, kShadeFD = 2, kShadePred = 3, kShadeAdj = 4 };

// Waves per workgroup cap (sets the VGPR budget through the launch bounds):
// value-mode networks with the packed FP16 latent path fit 4 waves per SIMD
// (<= 128 VGPRs), other value-mode networks 3 (<= 168). Forward mode: 3 for
// the c = 32 and c = 48 FP16 networks on a packed grid (spills of a few
// registers; with the persistent launch the third wave hides more than the
// spills cost: c = 48 measured 122 -> 106 ms per frame), 2 otherwise.
// Central differences add the neighbour offsets and the gradient gather to
// the value-mode network; with F = 16 channels gathered in FP32 (c = 48, or
// an FP16 network on an FP32 grid) that needs 2 waves per SIMD, c = 48 with
// the packed latent path 3. The adjoint keeps every layer's activation
// derivatives of two N-tiles in registers: 3 waves per SIMD for the c = 32
// FP16 network on a packed grid (151 -> 138 ms on the study views), 2
// otherwise (c = 48 measured 47 -> 48 ms at 3).
// FP32 networks add the FP64 ray of their sample positions (about 10
// registers).
template <class CF, int MODE, bool POINTS = false>
constexpr int max_waves() {
  if (MODE == kShadeAdj) return (CF::P == kF16 && CF::C == 32 && CF::G16) ? 12 : 8;
  if (MODE == kShadeFwd) return (CF::P == kF16 && CF::C <= 48 && CF::G16) ? 12 : 8;
  if (MODE == kShadeFD) {
    if (CF::F == 16 && (CF::C == 48 || (CF::P != kF32 && !CF::G16))) return 8;
    return (CF::G16 && CF::C == 32) ? 16 : 12;
  }
  // FP32 c = 48 network with F = 16: the FP64 sample positions need a few
  // more registers than 168
  if (CF::P == kF32 && CF::C == 48 && CF::F == 16) return 8;
  // point evaluation on an FP16 grid holds the corners over the feature build
  if (POINTS && CF::GK == 1) return 12;
  return CF::G16 ? 16 : 12;
}

// Render tile geometry per shading mode: lanes per ray and tile edges.
template <int MODE>
struct TileShape {
  static constexpr int LPR = (MODE == kShadeFwd) ? 4 : (MODE == kShadeFD ? 8 : 1);
  static constexpr int TW = LPR == 1 ? 8 : 4;
  static constexpr int TH = 64 / LPR / TW;
};
constexpr int kLdsBytes = 160 * 1024;

// LDS bytes of a workgroup besides its waves' input tiles: the forward weight
// fragments, and for the adjoint the transposed ones.
template <class CF, int MODE>
__host__ __device__ int fixed_lds_bytes(int H) {
  using G = typename CF::G;
  return G::weight_bytes(H) + (MODE == kShadeAdj ? G::back_bytes(H) : 0);
}

// Waves per workgroup. The VGPR budget of max_waves allows that many waves
// on a CU; every workgroup holds the weights once plus one input tile per
// wave in LDS. Pick the size that puts the most waves on a CU and, among
// sizes that reach it, the smallest: several smaller workgroups per CU let
// the dispatcher replace a finished one while another still runs its long
// rays (measured: 3 x 4 waves beat 1 x 12 waves by 12% on the BF16 path).
template <class CF, int MODE, bool POINTS = false>
int waves_per_block(int H) {
  using G = typename CF::G;
  constexpr int cap = max_waves<CF, MODE, POINTS>();
  const int wb = fixed_lds_bytes<CF, MODE>(H);
  int best = 0, best_waves = 0;
  for (int w = 1; w <= cap; ++w) {
    const int per_cu = kLdsBytes / (wb + w * G::FEAT_BYTES);
    const int waves = per_cu * w < cap ? per_cu * w : cap;
    if (per_cu >= 1 && waves > best_waves) {
      best = w;
      best_waves = waves;
    }
  }
  return best;
}

// Workgroups of wpb waves and shm bytes of LDS that the GPU holds at once (by
// LDS and by the VGPR budget of max_waves).
template <class CF, int MODE, bool POINTS = false>
long long resident_blocks(int wpb, size_t shm) {
  const int per_cu_lds = (int)(kLdsBytes / shm), per_cu_regs = max_waves<CF, MODE, POINTS>() / wpb;
  return (long long)device_cus() * (per_cu_lds < per_cu_regs ? per_cu_lds : per_cu_regs);
}

// ----------------------------------------------------- TF, camera, march

__device__ inline void tf_eval(const TFDev& tf, float d, float rgba[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) rgba[q] = tf.base[q];
  for (int j = 0; j < tf.n_seg; ++j) {
    const float w = __builtin_amdgcn_fmed3f(fmaf(d, tf.inv[j], tf.off[j]), 0.0f, 1.0f);
#pragma unroll
    for (int q = 0; q < 4; ++q) rgba[q] = fmaf(w, tf.delta[j][q], rgba[q]);
  }
}

// Segment i of a ray: midpoint parameter and length, the segment ending at
// t_end (the chord's end, or +inf for fixed-count marches: the last of their
// equal segments already ends there).
__device__ inline void segment(const Ray& r, int i, float t_end, float& tm, float& len) {
  const float a0 = fmaf((float)i, r.ds, r.t0);
  len = fminf(a0 + r.ds, t_end) - a0;
  tm = fmaf(0.5f, len, a0);
}

// Headlight Blinn-Phong (Sec. 6): light and view along -dir, normal = the
// normalized density gradient.
__device__ inline void phong(float rgba[4], float gx, float gy, float gz, const float dir[3], const MarchDev& m) {
  const float g2 = gx * gx + gy * gy + gz * gz;
  if (g2 >= 1e-12f) {  // |g| >= 1e-6
    // |n . l| with n = g / |g| by the hardware reciprocal square root, and
    // |n . l|^shininess as exp2(shininess * log2(.)) on the hardware
    // transcendentals (the library sqrt, divide and powf cost about 200
    // instructions per sample); the floor keeps log2 finite, so 0^0 = 1
    const float ndl = fabsf(gx * dir[0] + gy * dir[1] + gz * dir[2]) * __builtin_amdgcn_rsqf(g2);
    const float spec = m.ks * __builtin_amdgcn_exp2f(m.shininess * __builtin_amdgcn_logf(fmaxf(ndl, 1e-30f)));
    const float k = m.ka + m.kd * ndl;
    rgba[0] = fmaf(rgba[0], k, spec);
    rgba[1] = fmaf(rgba[1], k, spec);
    rgba[2] = fmaf(rgba[2], k, spec);
  }
}

// Front-to-back compositing of one segment (exact Beer-Lambert).
struct Accum {
  float T, C[3], A;
};

__device__ inline void composite(Accum& acc, const float rgba[4], float len) {
  const float trn = fast_exp(-rgba[3] * len);
  const float ta = acc.T * (1.0f - trn);
  acc.C[0] = fmaf(ta, rgba[0], acc.C[0]);
  acc.C[1] = fmaf(ta, rgba[1], acc.C[1]);
  acc.C[2] = fmaf(ta, rgba[2], acc.C[2]);
  acc.A += ta;
  acc.T *= trn;
}

// ------------------------------------------------------------- kernels

// Persistent: as many workgroups as the CUs hold at once, each wave taking
// tiles from a device-wide counter until none is left (queue[0]: the next
// tile; queue[1]: waves done, so that the last one sets both back to zero).
// Tile costs vary (empty, short and long rays): a static share of tiles per
// wave was measured 30% slower, and one tile per wave keeps a workgroup's
// LDS until its slowest wave ends, so the CUs ran at two thirds of their
// wave slots on average.
// HH: the network's layer count, compiled in for the adjoint (its saved
// activation derivatives are registers); 0 for the other modes.
template <class CF, int MODE, int HH = 0>
__global__ __launch_bounds__((max_waves<CF, MODE>() * 64)) void march_kernel(NetDev nd, TFDev tf, ViewBatch vb,
                                                                                  MarchDev m, float* out,
                                                                                  unsigned long long* stats,
                                                                                  unsigned int* queue,
                                                                                  int tiles_x, int tiles_y) {
  using G = typename CF::G;
  using E = typename CF::E;
  constexpr bool GRAD = MODE == kShadeFwd;  // network run in forward (tangent) mode
  constexpr bool FD = MODE == kShadeFD;
  constexpr int LPR = TileShape<MODE>::LPR, TW = TileShape<MODE>::TW;
  constexpr bool ADJ = MODE == kShadeAdj;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  stage_weights<CF>(nd, smem);
  char* bsm = smem + G::weight_bytes(nd.H);  // transposed fragments (adjoint)
  if constexpr (ADJ) stage_backward_adj<CF>(nd, bsm);
  __syncthreads();
  // the wave index is wave-uniform; saying so keeps the tile, its camera and
  // the latent grid's buffer resource in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int tiles_per_view = tiles_x * tiles_y;
  const int n_tiles = tiles_per_view * vb.n_views;
  const int rl = lane / LPR;  // ray within the tile
  const int q = lane % LPR;   // role of the lane within its ray
  const LaneRole role = GRAD ? grad_role(q) : value_role();
  // central differences: lane q = 1..6 evaluates the sample moved by +-h along
  // axis (q-1)/2 (odd q: +h); q = 0 and 7 evaluate the sample itself
  const float fh = (q & 1) ? m.fd_step : -m.fd_step;
  const float fd_off[3] = {FD && (q == 1 || q == 2) ? fh : 0.0f, FD && (q == 3 || q == 4) ? fh : 0.0f,
                           FD && (q == 5 || q == 6) ? fh : 0.0f};
  const float inv_2h = FD ? 0.5f / m.fd_step : 0.0f;
  const bool fixed = m.fixed_steps > 0;
  E* feat = reinterpret_cast<E*>(smem + fixed_lds_bytes<CF, MODE>(nd.H) + wave * G::FEAT_BYTES);
  E* myrow = feat + lane * G::ROW;
  unsigned long long n_samp = 0, n_hit = 0, iters = 0;
  for (int tile = next_tile(queue, lane); tile < n_tiles; tile = next_tile(queue, lane)) {
    const int v = tile / tiles_per_view;
    const int tr = tile % tiles_per_view;
    const int px = (tr % tiles_x) * TW + (rl % TW);
    const int py = (tr / tiles_x) * TileShape<MODE>::TH + (rl / TW);
    const CamDev& cam = vb.cam[v];
    const LatentSrc ls = make_latent_src(nd, cam.key, cam.key_w);
    const bool in_img = px < vb.width && py < vb.height;
    // FP32 networks take every sample position from the FP64 ray, rounded
    // once: an FP32 o + t d (the eye a few units from the box) is off by a
    // few 1e-7, which the highest Fourier octaves turn into visible density
    // and shading-normal errors; FP16/BF16 rounding dwarfs it
    constexpr bool kPosF64 = CF::P == kF32;
    const RayD rayd = make_ray_d(cam, in_img ? px : 0, in_img ? py : 0, vb.width, vb.height, m);
    const Ray ray = round_ray(rayd);
    bool active = in_img && ray.hit && ray.nseg > 0;
    float tfe[G::TIN > 0 ? G::TIN : 1];  // the view's time inputs (time-encoded networks)
    if constexpr (G::TIN > 0) time_features<CF::TE>(cam.tau, tfe);
    Accum acc = {1.0f, {0.0f, 0.0f, 0.0f}, 0.0f};
    const float t_end = fixed ? INFINITY : ray.t1;
    // position and length of segment ii. A lane whose ray has ended keeps
    // sampling its (finite) ray past the end: the cell clamps keep its loads
    // inside the grid and its result is not composited. The FP64 positions
    // of FP32 networks are zeroed for such lanes.
    auto sample_at = [&](int ii, bool act, float& sx, float& sy, float& sz, float& len) {
      if constexpr (kPosF64) {
        float pp[3];
        segment_d(rayd, ii, fixed, fd_off, pp, len);
        sx = act ? pp[0] : 0.0f;
        sy = act ? pp[1] : 0.0f;
        sz = act ? pp[2] : 0.0f;
      } else {
        float tm;
        segment(ray, ii, t_end, tm, len);
        sx = fmaf(tm, ray.d[0], ray.o[0]);
        sy = fmaf(tm, ray.d[1], ray.o[1]);
        sz = fmaf(tm, ray.d[2], ray.o[2]);
        if constexpr (FD) {
          sx += fd_off[0];
          sy += fd_off[1];
          sz += fd_off[2];
        }
      }
    };
    int i = 0;
    while (__builtin_amdgcn_ballot_w64(active)) {
      ++iters;
      float len, sx, sy, sz;
      sample_at(i, active, sx, sy, sz, len);
      write_features<CF, GRAD>(myrow, ls, role, sx, sy, sz, tfe, nd.fm);
      wave_lds_sync();
      f4 yo;
      float ga[3] = {0.0f, 0.0f, 0.0f};
      if constexpr (ADJ) {
        // the network and its adjoint; each row then holds dy/d(input row)
        yo[0] = mlp_tile_adj<CF, HH>(smem, bsm, feat);
        wave_lds_sync();
        input_vjp<CF>(myrow, ls, sx, sy, sz, ga);
      } else {
        yo = mlp_tile<CF, GRAD>(smem, feat, nd.H, role);
      }
      wave_lds_sync();
      const float y = yo[0];
      float dens, gx = 0.0f, gy = 0.0f, gz = 0.0f;
      if constexpr (ADJ) {
        dens = sigmoid_f(y);
        const float sg = dens * (1.0f - dens);
        gx = sg * ga[0];
        gy = sg * ga[1];
        gz = sg * ga[2];
      } else if constexpr (MODE == kShadePred) {
        // outputs 1..3 are the gradient itself
        dens = sigmoid_f(y);
        gx = yo[1];
        gy = yo[2];
        gz = yo[3];
      } else if constexpr (GRAD) {
        // the quad's value lane holds the logit, lanes 1..3 its derivatives
        const float y0 = quad_bcast0(y);
        const float t1 = quad_bcast<1>(y), t2 = quad_bcast<2>(y), t3 = quad_bcast<3>(y);
        dens = sigmoid_f(y0);
        const float sg = dens * (1.0f - dens);
        gx = sg * t1;
        gy = sg * t2;
        gz = sg * t3;
      } else if constexpr (FD) {
        // gather the seven densities of the ray's lane group
        const float dl = sigmoid_f(y);
        const int b = lane & ~7;
        dens = __shfl(dl, b, 64);
        gx = (__shfl(dl, b + 1, 64) - __shfl(dl, b + 2, 64)) * inv_2h;
        gy = (__shfl(dl, b + 3, 64) - __shfl(dl, b + 4, 64)) * inv_2h;
        gz = (__shfl(dl, b + 5, 64) - __shfl(dl, b + 6, 64)) * inv_2h;
      } else {
        dens = sigmoid_f(y);
      }
      // branch-free: a lane without a sample composites a zero-length
      // segment, which changes nothing (transmittance factor exp(0) = 1)
      const bool comp = active && len > 0.0f;
      float rgba[4];
      tf_eval(tf, dens, rgba);
      if (m.phong) phong(rgba, gx, gy, gz, ray.d, m);
      composite(acc, rgba, comp ? len : 0.0f);
      i += comp ? 1 : 0;
      active = comp && !(acc.T < m.ert_eps) && i < ray.nseg;
    }
    const bool owner = q == 0;
    if (in_img && owner) {
      float4* o = reinterpret_cast<float4*>(out) + ((long long)v * vb.height + py) * vb.width + px;
      *o = make_float4(acc.C[0], acc.C[1], acc.C[2], acc.A);
    }
    n_samp += owner ? (unsigned long long)i : 0ull;
    n_hit += (owner && in_img && ray.hit && ray.nseg > 0) ? 1ull : 0ull;
  }
  if (stats) {
    for (int off = 32; off > 0; off >>= 1) {
      n_samp += __shfl_xor(n_samp, off, 64);
      n_hit += __shfl_xor(n_hit, off, 64);
    }
    if (lane == 0 && (n_samp | n_hit | iters)) {
      atomicAdd(stats, n_samp);
      atomicAdd(stats + 1, n_hit);
      atomicAdd(stats + 2, iters * (unsigned long long)(64 / LPR));
    }
  }
  release_queue(queue, lane, gridDim.x * wpb);
}

// Point evaluation (PM): kShadeNone -- density, and with out_g set outputs
// 1..3 of a 4-output network (its predicted gradient); kShadeFwd -- density
// and forward-mode gradient; kShadeAdj -- density and adjoint gradient (HH:
// layer count, as for the render kernel).
template <class CF, int PM, int HH = 0>
__global__ __launch_bounds__((max_waves<CF, PM, true>() * 64)) void points_kernel(NetDev nd, const float* xyz, long long n,
                                                                            int key, float key_w, float* out_d,
                                                                            float* out_g) {
  using G = typename CF::G;
  using E = typename CF::E;
  constexpr bool GRAD = PM == kShadeFwd;
  constexpr bool ADJ = PM == kShadeAdj;
  constexpr int PER = GRAD ? 16 : 64;  // points per wave step
  extern __shared__ __attribute__((aligned(16))) char smem[];
  stage_weights<CF>(nd, smem);
  char* bsm = smem + G::weight_bytes(nd.H);
  if constexpr (ADJ) stage_backward_adj<CF>(nd, bsm);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  E* feat = reinterpret_cast<E*>(smem + fixed_lds_bytes<CF, PM>(nd.H) + wave * G::FEAT_BYTES);
  E* myrow = feat + lane * G::ROW;
  const LaneRole role = GRAD ? grad_role(lane & 3) : value_role();
  const LatentSrc ls = make_latent_src(nd, key, key_w);
  float tfe[G::TIN > 0 ? G::TIN : 1];  // time inputs of the evaluation time
  if constexpr (G::TIN > 0) time_features<CF::TE>(nd.tau, tfe);
  const long long nchunks = (n + PER - 1) / PER;
  const int waves = blockDim.x >> 6;
  const long long stride = (long long)gridDim.x * waves;
  // The next chunk's positions are read once this chunk's input rows are
  // built: the HBM read then runs behind this chunk's MLP instead of in
  // series with the latent gather that it addresses.
  float nx = 0.0f, ny = 0.0f, nz = 0.0f;
  auto load_pos = [&](long long cc) {
    const long long j = cc * PER + (GRAD ? (lane >> 2) : lane);
    nx = ny = nz = 0.0f;
    if (cc < nchunks && j < n) {
      nx = xyz[3 * j];
      ny = xyz[3 * j + 1];
      nz = xyz[3 * j + 2];
    }
  };
  long long c = (long long)blockIdx.x * waves + wave;
  load_pos(c);
  for (; c < nchunks; c += stride) {
    const long long idx = c * PER + (GRAD ? (lane >> 2) : lane);
    const bool ok = idx < n;
    const float x = nx, y = ny, z = nz;
    write_features<CF, GRAD, CF::P != kF32 && CF::GK == 1 && !GRAD>(myrow, ls, role, x, y, z, tfe, nd.fm);
    wave_lds_sync();
    load_pos(c + stride);
    if constexpr (ADJ) {
      const float o = mlp_tile_adj<CF, HH>(smem, bsm, feat);
      wave_lds_sync();
      float ga[3] = {0.0f, 0.0f, 0.0f};
      input_vjp<CF>(myrow, ls, x, y, z, ga);
      wave_lds_sync();
      const float d = sigmoid_f(o), sg = d * (1.0f - d);
      if (ok) {
        if (out_d) out_d[idx] = d;
        out_g[3 * idx] = sg * ga[0];
        out_g[3 * idx + 1] = sg * ga[1];
        out_g[3 * idx + 2] = sg * ga[2];
      }
      continue;
    }
    const f4 oo = mlp_tile<CF, GRAD>(smem, feat, nd.H, role);
    wave_lds_sync();
    const float o = oo[0];
    if constexpr (GRAD) {
      const float d = sigmoid_f(quad_bcast0(o));
      if (ok) {
        if (role.is_val) {
          if (out_d) out_d[idx] = d;
        } else {
          out_g[3 * idx + role.axis] = d * (1.0f - d) * o;
        }
      }
    } else if (ok) {
      if (out_d) out_d[idx] = sigmoid_f(o);
      if (out_g) {
        out_g[3 * idx] = oo[1];
        out_g[3 * idx + 1] = oo[2];
        out_g[3 * idx + 2] = oo[3];
      }
    }
  }
}

// ------------------------------------------------------------ launchers

template <class CF, int MODE, int HH = 0>
int launch_render_t(const NetDev& nd, const TFDev& tf, const ViewBatch& vb, const MarchDev& m, float* out,
                    unsigned long long* stats, hipStream_t st) {
  using G = typename CF::G;
  constexpr int TW = TileShape<MODE>::TW, TH = TileShape<MODE>::TH;
  const int tx = (vb.width + TW - 1) / TW, ty = (vb.height + TH - 1) / TH;
  const long long tiles = (long long)tx * ty * vb.n_views;
  if (tiles > 0x7fffffffLL) return kLaunchTooLarge;
  const int wpb = waves_per_block<CF, MODE>(nd.H);
  if (wpb < 1) return kLaunchNoLds;
  const size_t shm = (size_t)fixed_lds_bytes<CF, MODE>(nd.H) + (size_t)wpb * G::FEAT_BYTES;
  // the workgroups the CUs hold at once, fewer for small launches
  const long long resident = resident_blocks<CF, MODE>(wpb, shm);
  const long long want = (tiles + wpb - 1) / wpb;
  const long long blocks = want < resident ? want : resident;
  if (blocks < 1) return 0;
  unsigned int* queue = tile_queue_slot();
  if (!queue) return 2;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)march_kernel<CF, MODE, HH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    attr = true;
  }
  hipLaunchKernelGGL((march_kernel<CF, MODE, HH>), dim3((unsigned)blocks), dim3(wpb * 64), shm, st, nd, tf, vb, m,
                     out, stats, queue, tx, ty);
  return check_launch();
}

template <class CF, int PM, int HH = 0>
int launch_points_t(const NetDev& nd, const float* xyz, long long n, int key, float key_w, float* out_d,
                    float* out_g, hipStream_t st) {
  using G = typename CF::G;
  constexpr int PER = PM == kShadeFwd ? 16 : 64;
  const int wpb = waves_per_block<CF, PM, true>(nd.H);
  if (wpb < 1) return kLaunchNoLds;
  const size_t shm = (size_t)fixed_lds_bytes<CF, PM>(nd.H) + (size_t)wpb * G::FEAT_BYTES;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)points_kernel<CF, PM, HH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    attr = true;
  }
  // persistent: the workgroups the GPU holds at once walk the chunks (equal
  // cost), so the weights are staged once per workgroup and no workgroup
  // waits for another to release its LDS
  const int blocks = grid_blocks((n + PER - 1) / PER, wpb, (int)resident_blocks<CF, PM, true>(wpb, shm));
  hipLaunchKernelGGL((points_kernel<CF, PM, HH>), dim3(blocks), dim3(wpb * 64), shm, st, nd, xyz, n, key, key_w,
                     out_d, out_g);
  return check_launch();
}

}  // namespace

}  // namespace fvsrn_detail
