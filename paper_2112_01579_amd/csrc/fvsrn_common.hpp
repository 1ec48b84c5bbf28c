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

}  // namespace fvsrn_detail
