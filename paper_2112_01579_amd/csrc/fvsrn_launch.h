// Internal launch interface between the C ABI (fvsrn_api.cpp) and the gfx950
// kernels (fvsrn_kernels.hip). Host-side structs are plain data; everything
// the kernels need is precomputed here once per call.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace fvsrn_detail {

constexpr int kMaxViewsPerLaunch = 16;
constexpr int kMaxKeyframes = 64;
constexpr int kMaxDrawGrids = 64;  // error grids per batched weighted draw
constexpr int kMaxFourierRows = 24;  // 3L for L <= 8

// Keyframe times for per-point keyframe selection in training.
struct KeyTimes {
  int K;
  float t[kMaxKeyframes];
};
constexpr int kMaxTFPoints = 16;

// Transfer function in telescoping form: f(d) = base + sum_j
// clamp(d * inv_j + off_j, 0, 1) * delta_j; alpha already multiplied by the
// opacity scale (so the fourth channel is the extinction kappa).
struct TFDev {
  int n_seg;
  float base[4];
  float inv[kMaxTFPoints - 1];
  float off[kMaxTFPoints - 1];
  float delta[kMaxTFPoints - 1][4];
};

// Camera with its orthonormal basis precomputed on the host (FP64: each ray
// is set up in FP64 and rounded once, see ray_setup).
struct CamDev {
  double fwd[3], right[3], up[3];
  double tan_half, half_extent, aspect;
  float eye[3];
  int ortho;
  int key;        // first keyframe of the latent blend
  float key_w;    // weight of keyframe key + 1
  float tau;      // normalised time of the view (time-encoded networks)
};

struct MarchDev {
  float step;
  int fixed_steps;
  float ert_eps;
  int phong;
  float ka, kd, ks, shininess;
  int grad_mode;  // 0 forward mode, 1 central differences (network renders)
  float fd_step;
};

struct NetDev {
  const void* latent;
  const float* weights;
  int R, F, K, L, C, H, act, grid_f16;
  long long key_stride;  // elements between keyframe grids
  int grid_u8;           // uint8 codes; dequant holds (offset, scale) [K][F][2]
  const float* dequant;
  int NO;                // outputs: 1 (density) or 4 (density, predicted gradient)
  int time_enc;          // time inputs (Sec. 8): 0 none, 1 direct, 2 Fourier, 3 both
  float t_lo, t_hi, t_scale;  // normalisation of times: tau = (clamp(t) - t_lo) t_scale - 1
  float tau;             // normalised time of a point evaluation
  int fmat;              // Fourier features from fm (random Fourier features) instead of octaves
  float fm[kMaxFourierRows][3];  // rows of the Fourier matrix, revolutions per world unit
};

struct ViewBatch {
  int n_views, width, height;
  CamDev cam[kMaxViewsPerLaunch];
};

enum Prec { kF32 = 0, kF16 = 1, kBF16 = 2, kU8 = 3 };

// All launchers return 0 on success, 1 if the configuration is not compiled,
// 2 on a HIP launch error. `stream` is a hipStream_t.
int launch_render(const NetDev& net, int prec, const TFDev& tf, const ViewBatch& views,
                  const MarchDev& m, float* out, unsigned long long* stats, void* stream);
// A non-null out_g receives the gradient by gmode: 0 forward mode, 2 outputs
// 1..3 of a 4-output network (value mode), 3 the adjoint.
int launch_points(const NetDev& net, int prec, const float* xyz, long long n, int key,
                  float key_w, float* out_d, float* out_g, int gmode, void* stream);
int launch_render_dense(const float* vol, int nx, int ny, int nz, const TFDev& tf,
                        const ViewBatch& views, const MarchDev& m, float* out,
                        unsigned long long* stats, void* stream);
// out nullable; out_g (nullable) receives one-voxel central differences
int launch_dense_points(const float* vol, int nx, int ny, int nz, const float* xyz, long long n,
                        float* out, float* out_g, void* stream);
int launch_sample_points(uint64_t seed, uint64_t counter, long long n, float* xyz, void* stream);
int launch_cast(const float* src, void* dst, long long count, int dst_dtype, void* stream);
int launch_ssim(const float* a, const float* b, int width, int height, int n_images, float* out, void* stream);
int launch_quantize(const float* src, long long n, int channels, unsigned char* codes, float* dequant, void* stream);
// Adaptive resampling (Sec. 5.4): error-grid positions, the per-voxel mean
// absolute error, and positions drawn in proportion to an error grid.
int launch_voxel_points(uint64_t seed, uint64_t counter, int G, int per_voxel, float* xyz, void* stream);
int launch_error_reduce(const float* d, const float* vol, int nx, int ny, int nz, const float* xyz,
                        long long n_voxels, int per_voxel, float* E, void* stream);
size_t weighted_points_workspace_bytes(long long n_voxels);
int launch_weighted_points(uint64_t seed, uint64_t counter, const float* E, int G, long long n, float* xyz,
                           void* workspace, void* stream);
int launch_weighted_points_multi(uint64_t seed, uint64_t counter, int G, int n_grids, const int64_t* n_per_grid,
                                 float* xyz, const void* workspace, size_t stride, void* stream);

// Training (FP32). Workspace layout is owned by the kernels file.
size_t train_workspace_bytes(const NetDev& net, long long n);
int launch_train(const NetDev& net, const KeyTimes& kt, float* latent, float* weights, float* d_latent,
                 float* d_weights, const float* xyz, const float* times, long long n, const float* target,
                 const float* target_grad, float grad_weight, const float* dloss_dy, int use_adam, float lr_grid, float lr_mlp, float beta1, float beta2,
                 float eps, int step, float* m_lat, float* v_lat, float* m_w, float* v_w, float* out_loss,
                 void* workspace, size_t ws_bytes, int half, void* stream);

// Size of the per-GPU training workspace of fvsrn_train_step_noalloc.
constexpr size_t kStaticTrainScratchBytes = (size_t)96 << 20;
// Device address of that workspace on the current device (looked up once per
// device): 0, or 2 when the lookup fails.
int static_train_scratch(void** ptr);

const char* last_hip_error();

// Launcher results: 0 launched; 1 configuration not compiled; 2 the launch
// failed (last_hip_error); kLaunchNoLds the network's weight fragments leave
// no room for a wave's input tile in LDS; kLaunchTooLarge the work exceeds
// a 32-bit grid.
constexpr int kLaunchNoLds = 3;
constexpr int kLaunchTooLarge = 4;

// Shared host helpers (defined in fvsrn_misc.hip).
int check_launch();                                   // 0 or 2 after a launch
int grid_blocks(long long work, int per_block, int cap);
int device_cus();
// Dynamic tile queue of the render launches: a pair of counters [next tile,
// waves done] on the current device, zero when handed out (the launch that
// uses it sets it back to zero as its last wave ends). Calls rotate over
// kTileQueueSlots pairs, so up to that many render launches may be in flight
// on one device at once. nullptr when the device's counters cannot be
// located (last_hip_error).
constexpr int kTileQueueSlots = 1024;
unsigned int* tile_queue_slot();

// Per-precision network launchers (fvsrn_march.hip compiled per precision).
int launch_render_p0(const NetDev&, const TFDev&, const ViewBatch&, const MarchDev&, float*, unsigned long long*,
                     void*);
int launch_render_p1(const NetDev&, const TFDev&, const ViewBatch&, const MarchDev&, float*, unsigned long long*,
                     void*);
int launch_render_p2(const NetDev&, const TFDev&, const ViewBatch&, const MarchDev&, float*, unsigned long long*,
                     void*);
int launch_points_p0(const NetDev&, const float*, long long, int, float, float*, float*, int, void*);
int launch_points_p1(const NetDev&, const float*, long long, int, float, float*, float*, int, void*);
int launch_points_p2(const NetDev&, const float*, long long, int, float, float*, float*, int, void*);

// Adjoint-gradient render and points (fvsrn_adjoint.hip, FP32, FP16 and BF16
// networks).
#define FV_DECL_ADJ(P)                                                                                         \
  int launch_render_adj_p##P(const NetDev&, const TFDev&, const ViewBatch&, const MarchDev&, float*,          \
                             unsigned long long*, void*);                                                       \
  int launch_points_adj_p##P(const NetDev&, const float*, long long, int, float, float*, float*, void*);
// Networks with a Fourier matrix (fvsrn_rff.hip) and with a time encoding
// (fvsrn_time.hip), sine activation: unshaded render and point densities
// (FP32, FP16, BF16), forward-mode gradients and Phong (FP32, FP16); out_g
// nullable, gmode as for launch_points.
#define FV_DECL_XF(NAME, P)                                                                                    \
  int launch_render_##NAME##_p##P(const NetDev&, const TFDev&, const ViewBatch&, const MarchDev&, float*,     \
                                  unsigned long long*, void*);                                                  \
  int launch_points_##NAME##_p##P(const NetDev&, const float*, long long, int, float, float*, float*, int, void*);
FV_DECL_ADJ(0) FV_DECL_ADJ(1) FV_DECL_ADJ(2)
FV_DECL_XF(rff, 0) FV_DECL_XF(rff, 1) FV_DECL_XF(rff, 2)
FV_DECL_XF(time, 0) FV_DECL_XF(time, 1) FV_DECL_XF(time, 2)
#undef FV_DECL_ADJ
#undef FV_DECL_XF

}  // namespace fvsrn_detail
