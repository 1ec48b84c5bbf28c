// Device-side building blocks shared by the gfx950 kernels: MFMA precision
// traits, the compile-time geometry of a network configuration, and small
// numeric helpers (revolution-based sine, clamped vertex-centred cells).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvsrn_launch.h"

namespace fvsrn_detail {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr float kInv2Pi = 0.15915494309189535f;
constexpr float k2Pi = 6.283185307179586f;
constexpr float kPi = 3.14159265358979323846f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kWave = 64;

enum Act { kSine = 0, kSnakeAlt = 1, kIdentity = 2 };

// ------------------------------------------------------------- precision

template <int P>
struct PrecT;

template <>
struct PrecT<kF16> {
  using E = _Float16;
  static constexpr int KC = 32;  // K of the main MFMA step
  static constexpr int KT = 8;   // input-row columns of the tail (x y z 1 0 0 0 0)
  using VA = h8;
  using VT = h4;
  __device__ static f4 mma(VA a, VA b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
  __device__ static f4 mmt(VT a, VT b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
};

template <>
struct PrecT<kBF16> {
  using E = __bf16;
  static constexpr int KC = 32;
  static constexpr int KT = 8;
  using VA = b8;
  using VT = b4;
  __device__ static f4 mma(VA a, VA b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  __device__ static f4 mmt(VT a, VT b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0,
                                                     0, 0);
  }
};

template <>
struct PrecT<kF32> {
  using E = float;
  static constexpr int KC = 4;
  static constexpr int KT = 4;
  using VA = float;
  using VT = float;
  __device__ static f4 mma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// Compile-time geometry of one network configuration (precision P, hidden
// width C, latent channels F, Fourier octaves L, time encoding TE).
//
// Layer 0's input row, one per sample, lives in LDS in the order
//   [latent F | sin 3L | cos 3L | zero pad to KMAIN | x y z 1 time | zero pad to KROW]
// so its first KF columns are the packed FP32 inputs 3.. in order and the
// constant-1 column carries the first layer's bias. The time inputs (Sec. 8)
// follow it: tau (direct), then sin and cos of pi 2^k tau, k < 4 (Fourier).
// For FP16/BF16 the tail (8 or 16 columns) is one K32 MFMA step whose A
// operand is zero beyond the used columns.
template <int P, int C, int F, int L, int TE = 0>
struct Geo {
  using PR = PrecT<P>;
  using E = typename PR::E;
  static constexpr int MT = C / 16;                       // M-tiles of a hidden layer
  static constexpr int KF = F + 6 * L;                    // latent + Fourier inputs
  static constexpr int TIN = TE == 0 ? 0 : (TE == 1 ? 1 : (TE == 2 ? 8 : 9));  // time inputs
  static constexpr int K0IN = 3 + KF + TIN;               // layer 0 inputs in the weight layout
  static constexpr int KMAIN = (KF + PR::KC - 1) / PR::KC * PR::KC;
  // tail: x y z 1 and the time inputs, rounded to the MFMA step's columns
  static constexpr int KT = (4 + TIN + PR::KT - 1) / PR::KT * PR::KT;
  static constexpr int KROW = KMAIN + KT;
  // input-row column of input k of the weight layout [x y z | latent | sin | cos | time]
  __host__ __device__ static constexpr int feat_col(int k) {
    return k < 3 ? KMAIN + k : (k < 3 + KF ? k - 3 : KMAIN + 4 + (k - 3 - KF));
  }
  static constexpr int S0 = KMAIN / PR::KC;               // main K steps of layer 0 (f16/bf16)
  static constexpr int Q0 = KROW / 4;                     // K4 steps of layer 0 (f32)
  // LDS row stride in dwords: the smallest >= the row with stride = 4 (mod 8),
  // so that 16-byte reads of 8 consecutive rows land on distinct banks
  static constexpr int RAW_DW = KROW * (int)sizeof(E) / 4;
  static constexpr int ROW_DW = RAW_DW + ((4 - RAW_DW % 8) + 8) % 8;
  static constexpr int ROW = ROW_DW * 4 / (int)sizeof(E);  // elements
  static constexpr int HS32 = MT / 2, HS16 = MT % 2;      // K steps of a hidden layer (f16/bf16)
  static constexpr bool kF32Path = (P == kF32);
  // byte sizes of the staged weight regions (A fragments in lane order)
  static constexpr int W0A = kF32Path ? MT * Q0 * kWave * 4 : MT * S0 * kWave * 16;
  static constexpr int W0T = kF32Path ? 0 : MT * kWave * 16;
  static constexpr int WHA = kF32Path ? MT * 4 * MT * kWave * 4 : MT * HS32 * kWave * 16;
  static constexpr int WHT = kF32Path ? 0 : MT * HS16 * kWave * 8;
  static constexpr int BH = C * 4;
  static constexpr int HID = WHA + WHT + BH;
  static constexpr int WOA = kF32Path ? 4 * 4 * MT * kWave * 4 : 4 * HS32 * kWave * 16;
  static constexpr int WOT = kF32Path ? 0 : 4 * HS16 * kWave * 8;
  static constexpr int BO = 16;
  __host__ __device__ static int weight_bytes(int H) { return W0A + W0T + (H - 1) * HID + WOA + WOT + BO; }
  // transposed (backward) fragments of the adjoint pass: W_i^T of each hidden
  // layer (same shape as W_i, no bias), W_0^T over MB0 16-row tiles covering
  // the input row's columns, and the output weights (FP32)
  static constexpr int MB0 = (KROW + 15) / 16;
  static constexpr int WBH = WHA + WHT;
  static constexpr int WB0A = kF32Path ? MB0 * 4 * MT * kWave * 4 : MB0 * HS32 * kWave * 16;
  static constexpr int WB0 = WB0A + (kF32Path ? 0 : MB0 * HS16 * kWave * 8);
  static constexpr int WOUT = C * 4;
  __host__ __device__ static int back_bytes(int H) { return (H - 1) * WBH + WB0 + WOUT; }
  static constexpr int FEAT_BYTES = kWave * ROW_DW * 4;  // one wave's input tile
};

// ------------------------------------------------------- small helpers

__device__ inline void wave_lds_sync() {
  // LDS operations of one wavefront complete in order; this only keeps the
  // compiler from moving reads of other lanes' rows across the writes.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Dynamic tile queue of a persistent launch: q[0] counts the tiles handed
// out, q[1] the waves that have finished. Called by every lane of a wave
// (wave-uniform result).
__device__ inline int next_tile(unsigned int* q, int lane) {
  unsigned int t = 0;
  if (lane == 0) t = atomicAdd(q, 1u);
  return (int)__builtin_amdgcn_readfirstlane(t);
}
// After a wave's last next_tile: counts it as done; the launch's last wave
// sets the pair back to zero for the next launch that uses it.
__device__ inline void release_queue(unsigned int* q, int lane, unsigned int total_waves) {
  if (lane == 0) {
    __threadfence();
    if (atomicAdd(q + 1, 1u) == total_waves - 1) {
      atomicExch(q, 0u);
      atomicExch(q + 1, 0u);
    }
  }
}

template <typename E>
__device__ inline E to_e(float x) {
  return (E)x;
}

__device__ inline float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }  // sin(2 pi r)
__device__ inline float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }  // cos(2 pi r)
__device__ inline float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ inline float sigmoid_f(float y) { return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-y * kLog2e)); }

// Value of lane 4*floor(lane/4) (the first lane of each quad). Called with
// every lane active; bound_ctrl lets the compiler fold the move into the
// instruction that consumes it as a DPP source operand.
__device__ inline float quad_bcast0(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x00, 0xF, 0xF, true));
}
// Value of lane 4*floor(lane/4) + k for k = 1, 2, 3.
template <int K>
__device__ inline float quad_bcast(float x) {
  constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), ctrl, 0xF, 0xF, false));
}

// Grid coordinate along one axis: vertex i at -1 + 2i/(R-1); the coordinate
// is clamped to the domain (derivative zero outside it) and the cell index
// capped at R-2. dfdp = d frac / d p.
__device__ inline void axis_cell(float p, int R, int& i, float& f, float& dfdp) {
  const float scale = 0.5f * (float)(R - 1);
  dfdp = (p < -1.0f || p > 1.0f) ? 0.0f : scale;
  // u = (p + 1) (R - 1) / 2 clamped to [0, R - 1]
  const float u = __builtin_amdgcn_fmed3f(fmaf(p, scale, scale), 0.0f, (float)(R - 1));
  int ii = (int)u;
  ii = ii > R - 2 ? R - 2 : ii;
  i = ii;
  f = u - (float)ii;
}

__device__ inline void axis_cell(float p, int R, int& i, float& f) {
  float d;
  axis_cell(p, R, i, f, d);
}

// axis_cell for the packed FP16 gathers: the coordinate is clamped to the
// float just below R-1, so its integer part is at most R-2 without a separate
// cap and its fraction is one v_fract (on the top face the fraction is then
// 1 - 2^-24 (R-1) instead of 1, far below the FP16 rounding of the weights).
__device__ inline void axis_cell_h(float p, int R, int& i, float& f, float& dfdp) {
  const float scale = 0.5f * (float)(R - 1);
  dfdp = (p < -1.0f || p > 1.0f) ? 0.0f : scale;
  const float top = __uint_as_float(__float_as_uint((float)(R - 1)) - 1u);
  const float u = __builtin_amdgcn_fmed3f(fmaf(p, scale, scale), 0.0f, top);
  i = (int)u;
  f = __builtin_amdgcn_fractf(u);
}

// Element offset of a vertex, x fastest: ix sx + iy sy + iz sz, the y and z
// terms on the 24-bit multipliers (every index and stride of a grid below
// 2^31 bytes fits 24 bits; sx is the channel count, a power of two).
__device__ inline unsigned vertex_offset(int ix, int iy, int iz, unsigned sx, unsigned sy, unsigned sz) {
  return __umul24((unsigned)iz, sz) + __umul24((unsigned)iy, sy) + (unsigned)ix * sx;
}

// ------------------------------------------------------------- rays

// One view ray: origin, unit direction, the chord [t0, t1] inside [-1,1]^3
// (t0 >= 0), the segment length and count; RayD in FP64, Ray rounded once.
struct RayD {
  double o[3], d[3];
  double t0, t1, ds;
  int nseg;
  bool hit;
};

struct Ray {
  float o[3], d[3];
  float t0, t1, ds;
  int nseg;
  bool hit;
};

// Ray of pixel (px, py), row 0 at the top, set up in FP64 (once per ray).
// Rounded once to FP32 (make_ray), a small direction component keeps its
// relative precision, where an FP32 set-up leaves it an absolute error that
// moves a grazing ray's entry into the box by up to that error over the
// component (1e-5 world units and more). Perspective rays start at the eye;
// orthographic rays at eye + h (aspect nx right + ny up), along forward.
// Fixed-step marches cut the chord into m.fixed_steps equal segments, others
// into ceil(chord / m.step) segments, the last one clipped at t1.
__device__ inline RayD make_ray_d(const CamDev& cam, int px, int py, int W, int H, const MarchDev& m) {
  RayD r;
  const double nx = (2.0 * px + 1.0) / (double)W - 1.0;
  const double ny = 1.0 - (2.0 * py + 1.0) / (double)H;
  const double sx = cam.aspect * nx;
  if (cam.ortho) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r.o[a] = (double)cam.eye[a] + cam.half_extent * (sx * cam.right[a] + ny * cam.up[a]);
      r.d[a] = cam.fwd[a];
    }
  } else {
    double l2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r.o[a] = cam.eye[a];
      r.d[a] = cam.fwd[a] + cam.tan_half * (sx * cam.right[a] + ny * cam.up[a]);
      l2 += r.d[a] * r.d[a];
    }
    const double inv = 1.0 / sqrt(l2);
#pragma unroll
    for (int a = 0; a < 3; ++a) r.d[a] *= inv;
  }
  double tn = -INFINITY, tf = INFINITY;
  bool miss = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (r.d[a] == 0.0) {
      if (r.o[a] < -1.0 || r.o[a] > 1.0) miss = true;
    } else {
      double ta = (-1.0 - r.o[a]) / r.d[a], tb = (1.0 - r.o[a]) / r.d[a];
      if (ta > tb) {
        const double s = ta;
        ta = tb;
        tb = s;
      }
      tn = fmax(tn, ta);
      tf = fmin(tf, tb);
    }
  }
  tn = fmax(tn, 0.0);
  r.hit = !miss && tf > tn;
  r.t0 = tn;
  r.t1 = r.hit ? tf : tn;
  if (m.fixed_steps > 0) {
    r.nseg = r.hit ? m.fixed_steps : 0;
    r.ds = (r.t1 - r.t0) / (double)m.fixed_steps;
  } else {
    r.ds = m.step;
    r.nseg = r.hit ? (int)ceil((r.t1 - r.t0) / (double)m.step) : 0;
  }
  return r;
}

__device__ inline Ray round_ray(const RayD& rd) {
  Ray r;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.o[a] = (float)rd.o[a];
    r.d[a] = (float)rd.d[a];
  }
  r.t0 = (float)rd.t0;
  r.t1 = (float)rd.t1;
  r.ds = (float)rd.ds;
  r.nseg = rd.nseg;
  r.hit = rd.hit;
  return r;
}

__device__ inline Ray make_ray(const CamDev& cam, int px, int py, int W, int H, const MarchDev& m) {
  return round_ray(make_ray_d(cam, px, py, W, H, m));
}

// Segment i of an FP64 ray: its midpoint (plus an offset `off`, world
// units) rounded once to FP32, and its length (the last one clipped).
__device__ inline void segment_d(const RayD& r, int i, bool fixed, const float off[3], float p[3], float& len) {
  const double a0 = r.t0 + (double)i * r.ds;
  double a1 = r.t0 + (double)(i + 1) * r.ds;
  if (!fixed) a1 = fmin(a1, r.t1);
  len = (float)(a1 - a0);
  const double tm = 0.5 * (a0 + a1);
#pragma unroll
  for (int a = 0; a < 3; ++a) p[a] = (float)(r.o[a] + tm * r.d[a] + (double)off[a]);
}

}  // namespace fvsrn_detail
