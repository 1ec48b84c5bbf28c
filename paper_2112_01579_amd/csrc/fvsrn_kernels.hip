// gfx950 kernels of the fV-SRN hot path.
//
// Work decomposition (one wavefront of 64 lanes is the unit everywhere):
//  * Each lane owns one ray (render) or one point (eval). Per march step the
//    lane builds its sample's network input -- trilinear latent vector
//    (Sec. 4.2), octave Fourier features (Sec. 3, Eq. 1-2), position and a
//    constant 1 that carries the first layer's bias -- and writes it as one
//    row of the wave's private LDS tile (64 rows).
//  * The MLP (Sec. 3) then runs on the matrix cores with samples on the N
//    axis of v_mfma_f32_16x16x32_{f16,bf16} (or 16x16x4_f32): 4 N-tiles of 16
//    samples per step. A D fragment leaves lane (g, n) holding output rows
//    4g..4g+3 of sample n; the next layer's weight columns are permuted when
//    the weights are staged so that those D values *are* the lane's B
//    fragment. Activations never leave registers between layers.
//  * The c -> 1 output layer is an MFMA whose A operand for N-tile t holds the
//    output weights in row 4t only. Summed over the 4 N-tiles into one
//    accumulator, row 4g of column n is the logit of sample (tile g, column
//    n), i.e. of the sample owned by lane 16g + n: no cross-lane reduction.
//  * Sine activations use v_sin_f32, which takes its argument in
//    revolutions; layers 0..H-1 are staged pre-multiplied by 1/(2 pi), so the
//    accumulator already holds revolutions.
//  * Weights are converted from the FP32 master copy into fragment order in
//    LDS once per workgroup; no buffer is allocated anywhere.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvsrn_launch.h"

namespace fvsrn_detail {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr float kInv2Pi = 0.15915494309189535f;
constexpr float kPi = 3.14159265358979323846f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kWave = 64;

// ------------------------------------------------------------- precision

template <int P>
struct PrecT;

template <>
struct PrecT<kF16> {
  using E = _Float16;
  static constexpr int KC = 32;  // K of the main MFMA step
  static constexpr int KT = 16;  // K of the tail step (position + bias column)
  using VA = h8;
  using VT = h4;
  __device__ static f4 mma(VA a, VA b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  __device__ static f4 mmt(VT a, VT b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct PrecT<kBF16> {
  using E = __bf16;
  static constexpr int KC = 32;
  static constexpr int KT = 16;
  using VA = b8;
  using VT = b4;
  __device__ static f4 mma(VA a, VA b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static f4 mmt(VT a, VT b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a),
                                                     __builtin_bit_cast(s4, b), c, 0, 0, 0);
  }
};

template <>
struct PrecT<kF32> {
  using E = float;
  static constexpr int KC = 4;
  static constexpr int KT = 4;
  using VA = float;
  using VT = float;
  __device__ static f4 mma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Compile-time geometry of one network configuration.
template <int P, int C, int F, int L>
struct Geo {
  using PR = PrecT<P>;
  using E = typename PR::E;
  static constexpr int MT = C / 16;                       // M-tiles of a hidden layer
  static constexpr int KF = F + 6 * L;                    // latent + Fourier inputs
  static constexpr int KMAIN = (KF + PR::KC - 1) / PR::KC * PR::KC;
  static constexpr int KROW = KMAIN + PR::KT;             // + [x, y, z, 1, 0...]
  static constexpr int S0 = KMAIN / PR::KC;               // main K steps of layer 0
  static constexpr int Q0 = KROW / 4;                     // FP32: K4 steps of layer 0
  // LDS row stride: 16-byte reads of 8 consecutive rows land on distinct banks
  static constexpr int ROW_DW = ((KROW * (int)sizeof(E) / 4 + 7) / 8) * 8 + 4;
  static constexpr int ROW = ROW_DW * 4 / (int)sizeof(E); // elements
  static constexpr int HS32 = MT / 2, HS16 = MT % 2;      // K steps of a hidden layer (f16/bf16)
  static constexpr bool kF32Path = (P == kF32);
  // byte sizes of the staged weight regions
  static constexpr int W0A = kF32Path ? MT * Q0 * kWave * 4 : MT * S0 * kWave * 16;
  static constexpr int W0T = kF32Path ? 0 : MT * kWave * 8;
  static constexpr int WHA = kF32Path ? MT * 4 * MT * kWave * 4 : MT * HS32 * kWave * 16;
  static constexpr int WHT = kF32Path ? 0 : MT * HS16 * kWave * 8;
  static constexpr int BH = C * 4;
  static constexpr int HID = WHA + WHT + BH;
  static constexpr int WOA = kF32Path ? 4 * 4 * MT * kWave * 4 : 4 * HS32 * kWave * 16;
  static constexpr int WOT = kF32Path ? 0 : 4 * HS16 * kWave * 8;
  static constexpr int BO = 16;
  __host__ __device__ static int weight_bytes(int H) { return W0A + W0T + (H - 1) * HID + WOA + WOT + BO; }
  static constexpr int FEAT_BYTES = kWave * ROW_DW * 4;   // one wave's input tile
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

__device__ inline float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ inline float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// Activation applied to an accumulator holding the pre-activation (in
// revolutions for the periodic activations).
__device__ inline float activate(float r, int act) {
  if (act == 0) return sin_rev(r);                 // sin(2 pi r)
  if (act == 1) {                                  // SnakeAlt(x) = x/2 + sin^2 x, x = 2 pi r
    float s = sin_rev(r);
    return fmaf(kPi, r, s * s);
  }
  return r;                                        // identity
}

__device__ inline float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }

__device__ inline float sigmoid_f(float y) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-y * kLog2e));
}

// Grid coordinate along one axis (vertex-centred, clamped, cell index <= R-2).
__device__ inline void axis_cell(float p, int R, int& i, float& f) {
  float u = (p + 1.0f) * 0.5f * (float)(R - 1);
  u = fminf(fmaxf(u, 0.0f), (float)(R - 1));
  int ii = (int)u;
  ii = ii > R - 2 ? R - 2 : ii;
  i = ii;
  f = u - (float)ii;
}

// Accumulate w * G[corner][0..F) into z.
template <int F>
__device__ inline void gather_corner(const void* grid, bool f16, long long idx, float w, float* z) {
  if (f16) {
    const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const _Float16*>(grid) + idx);
#pragma unroll
    for (int q = 0; q < F / 8; ++q) {
      uint4 v = src[q];
      h8 hv = __builtin_bit_cast(h8, v);
#pragma unroll
      for (int j = 0; j < 8; ++j) z[8 * q + j] = fmaf(w, (float)hv[j], z[8 * q + j]);
    }
  } else {
    const float4* src = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(grid) + idx);
#pragma unroll
    for (int q = 0; q < F / 4; ++q) {
      float4 v = src[q];
      z[4 * q + 0] = fmaf(w, v.x, z[4 * q + 0]);
      z[4 * q + 1] = fmaf(w, v.y, z[4 * q + 1]);
      z[4 * q + 2] = fmaf(w, v.z, z[4 * q + 2]);
      z[4 * q + 3] = fmaf(w, v.w, z[4 * q + 3]);
    }
  }
}

// Trilinear latent vector of one keyframe grid, scaled by `scale` and added to z.
template <int F>
__device__ inline void latent_trilinear(const NetDev& nd, int key, float scale, float px, float py,
                                        float pz, float* z) {
  const int R = nd.R;
  int ix, iy, iz;
  float fx, fy, fz;
  axis_cell(px, R, ix, fx);
  axis_cell(py, R, iy, fy);
  axis_cell(pz, R, iz, fz);
  const long long sx = F, sy = (long long)R * F, sz = (long long)R * R * F;
  const long long base = key * nd.key_stride + iz * sz + iy * sy + ix * sx;
  const bool f16 = nd.grid_f16 != 0;
  const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
  const float wz0 = gz * scale, wz1 = fz * scale;
  gather_corner<F>(nd.latent, f16, base, gx * gy * wz0, z);
  gather_corner<F>(nd.latent, f16, base + sx, fx * gy * wz0, z);
  gather_corner<F>(nd.latent, f16, base + sy, gx * fy * wz0, z);
  gather_corner<F>(nd.latent, f16, base + sx + sy, fx * fy * wz0, z);
  gather_corner<F>(nd.latent, f16, base + sz, gx * gy * wz1, z);
  gather_corner<F>(nd.latent, f16, base + sz + sx, fx * gy * wz1, z);
  gather_corner<F>(nd.latent, f16, base + sz + sy, gx * fy * wz1, z);
  gather_corner<F>(nd.latent, f16, base + sz + sx + sy, fx * fy * wz1, z);
}

// ------------------------------------------------------ weight staging

// Layer 0's LDS feature row order is [latent F | sin 3L | cos 3L | zero pad |
// x y z 1 | zero pad]; the packed FP32 input order is [x y z | latent | sin |
// cos], so the first KF columns are the packed inputs 3.. in order and the
// constant-1 column carries the bias.
template <int P, int C, int F, int L>
__device__ void stage_weights(const NetDev& nd, char* smem) {
  using G = Geo<P, C, F, L>;
  using E = typename G::E;
  constexpr int MT = G::MT;
  const int H = nd.H, K0 = 3 + F + 6 * L;
  const float* w = nd.weights;
  const float sc = nd.act == 2 ? 1.0f : kInv2Pi;
  const int tid = threadIdx.x, nt = blockDim.x;
  // offsets in the packed FP32 array
  const long long off_b0 = (long long)C * K0;
  auto off_hidden = [&](int i) -> long long {  // W_i for 1 <= i <= H
    return (long long)C * K0 + C + (long long)(i - 1) * (C * C + C);
  };
  auto w0 = [&](int o, int col) -> float {
    if (col < G::KF) return w[(long long)o * K0 + 3 + col] * sc;
    if (col < G::KMAIN) return 0.0f;
    const int t = col - G::KMAIN;
    if (t < 3) return w[(long long)o * K0 + t] * sc;
    if (t == 3) return w[off_b0 + o] * sc;
    return 0.0f;
  };
  char* p = smem;
  if constexpr (P == kF32) {
    float* W0 = reinterpret_cast<float*>(p);
    for (int e = tid; e < MT * G::Q0 * kWave; e += nt) {
      const int lane = e % kWave, q = (e / kWave) % G::Q0, mt = e / (kWave * G::Q0);
      const int g = lane >> 4, m = lane & 15;
      W0[e] = w0(16 * mt + m, g * G::Q0 + q);
    }
    p += G::W0A;
    for (int i = 1; i < H; ++i) {
      const float* Wi = w + off_hidden(i);
      float* WH = reinterpret_cast<float*>(p);
      for (int e = tid; e < MT * 4 * MT * kWave; e += nt) {
        const int lane = e % kWave, q = (e / kWave) % (4 * MT), mt = e / (kWave * 4 * MT);
        const int g = lane >> 4, m = lane & 15;
        const int ch = 16 * (q / 4) + 4 * g + (q % 4);
        WH[e] = Wi[(16 * mt + m) * C + ch] * sc;
      }
      float* BHp = reinterpret_cast<float*>(p + G::WHA);
      for (int e = tid; e < C; e += nt) BHp[e] = Wi[C * C + e] * sc;
      p += G::HID;
    }
    const float* Wo = w + off_hidden(H);
    float* WO = reinterpret_cast<float*>(p);
    for (int e = tid; e < 4 * 4 * MT * kWave; e += nt) {
      const int lane = e % kWave, q = (e / kWave) % (4 * MT), t = e / (kWave * 4 * MT);
      const int g = lane >> 4, m = lane & 15;
      const int ch = 16 * (q / 4) + 4 * g + (q % 4);
      WO[e] = (m == 4 * t) ? Wo[ch] : 0.0f;
    }
    p += G::WOA;
    if (tid == 0) *reinterpret_cast<float*>(p) = Wo[C];
  } else {
    E* W0A = reinterpret_cast<E*>(p);
    for (int e = tid; e < MT * G::S0 * kWave * 8; e += nt) {
      const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::S0, mt = (e >> 9) / G::S0;
      const int g = lane >> 4, m = lane & 15;
      W0A[e] = to_e<E>(w0(16 * mt + m, 32 * s + 8 * g + j));
    }
    E* W0T = reinterpret_cast<E*>(p + G::W0A);
    for (int e = tid; e < MT * kWave * 4; e += nt) {
      const int j = e & 3, lane = (e >> 2) & 63, mt = e >> 8;
      const int g = lane >> 4, m = lane & 15;
      W0T[e] = to_e<E>(w0(16 * mt + m, G::KMAIN + 4 * g + j));
    }
    p += G::W0A + G::W0T;
    for (int i = 1; i < H; ++i) {
      const float* Wi = w + off_hidden(i);
      E* WA = reinterpret_cast<E*>(p);
      for (int e = tid; e < MT * G::HS32 * kWave * 8; e += nt) {
        const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::HS32, mt = (e >> 9) / G::HS32;
        const int g = lane >> 4, m = lane & 15;
        const int ch = j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4);
        WA[e] = to_e<E>(Wi[(16 * mt + m) * C + ch] * sc);
      }
      if constexpr (G::HS16) {
        E* WT = reinterpret_cast<E*>(p + G::WHA);
        for (int e = tid; e < MT * kWave * 4; e += nt) {
          const int j = e & 3, lane = (e >> 2) & 63, mt = e >> 8;
          const int g = lane >> 4, m = lane & 15;
          const int ch = 16 * (MT - 1) + 4 * g + j;
          WT[e] = to_e<E>(Wi[(16 * mt + m) * C + ch] * sc);
        }
      }
      float* BHp = reinterpret_cast<float*>(p + G::WHA + G::WHT);
      for (int e = tid; e < C; e += nt) BHp[e] = Wi[C * C + e] * sc;
      p += G::HID;
    }
    const float* Wo = w + off_hidden(H);
    E* WOA = reinterpret_cast<E*>(p);
    for (int e = tid; e < 4 * G::HS32 * kWave * 8; e += nt) {
      const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::HS32, t = (e >> 9) / G::HS32;
      const int g = lane >> 4, m = lane & 15;
      const int ch = j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4);
      WOA[e] = to_e<E>(m == 4 * t ? Wo[ch] : 0.0f);
    }
    if constexpr (G::HS16) {
      E* WOT = reinterpret_cast<E*>(p + G::WOA);
      for (int e = tid; e < 4 * kWave * 4; e += nt) {
        const int j = e & 3, lane = (e >> 2) & 63, t = e >> 8;
        const int g = lane >> 4, m = lane & 15;
        const int ch = 16 * (MT - 1) + 4 * g + j;
        WOT[e] = to_e<E>(m == 4 * t ? Wo[ch] : 0.0f);
      }
    }
    p += G::WOA + G::WOT;
    if (tid == 0) *reinterpret_cast<float*>(p) = Wo[C];
  }
}

// ------------------------------------------------------ network input

// Builds this lane's input row (see w0 above for the column order) at
// position p and writes it to `row` in LDS.
template <int P, int C, int F, int L>
__device__ inline void write_features(typename Geo<P, C, F, L>::E* row, const NetDev& nd, int key,
                                      float key_w, float px, float py, float pz) {
  using G = Geo<P, C, F, L>;
  using E = typename G::E;
  float v[G::KROW];
#pragma unroll
  for (int j = 0; j < G::KROW; ++j) v[j] = 0.0f;
  // latent vector, blended between keyframes key and key + 1 (Sec. 8)
  if (nd.K > 1) {
    latent_trilinear<F>(nd, key, 1.0f - key_w, px, py, pz, v);
    latent_trilinear<F>(nd, key + 1, key_w, px, py, pz, v);
  } else {
    latent_trilinear<F>(nd, 0, 1.0f, px, py, pz, v);
  }
  // Fourier features: sin/cos(pi 2^k p) = sin/cos of 2^(k-1) p revolutions;
  // the power-of-two scaling is exact, so the phase carries no rounding.
  const float pp[3] = {px, py, pz};
#pragma unroll
  for (int k = 0; k < L; ++k) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float ph = pp[a] * (float)(1 << k) * 0.5f;
      v[F + 3 * k + a] = sin_rev(ph);
      v[F + 3 * L + 3 * k + a] = cos_rev(ph);
    }
  }
  v[G::KMAIN + 0] = px;
  v[G::KMAIN + 1] = py;
  v[G::KMAIN + 2] = pz;
  v[G::KMAIN + 3] = 1.0f;
  if constexpr (P == kF32) {
    float4* dst = reinterpret_cast<float4*>(row);
#pragma unroll
    for (int q = 0; q < G::KROW / 4; ++q)
      dst[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
    using V8 = typename PrecT<P>::VA;
    V8* dst = reinterpret_cast<V8*>(row);
#pragma unroll
    for (int q = 0; q < G::KROW / 8; ++q) {
      V8 x;
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = to_e<E>(v[8 * q + j]);
      dst[q] = x;
    }
  }
}

// ------------------------------------------------------------- the MLP

// Runs the network on the wave's 64 input rows. Returns the logit of the
// sample in this lane's own row.
template <int P, int C, int F, int L>
__device__ inline float mlp_tile(const char* wsm, const typename Geo<P, C, F, L>::E* feat, int H,
                                 int act) {
  using G = Geo<P, C, F, L>;
  using PR = PrecT<P>;
  using E = typename G::E;
  constexpr int MT = G::MT;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15;
  f4 out = {0.0f, 0.0f, 0.0f, 0.0f};
  if constexpr (P == kF32) {
    const float* W0 = reinterpret_cast<const float*>(wsm);
    for (int t = 0; t < 4; ++t) {
      f4 acc[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      const float* brow = feat + (16 * t + n) * G::ROW + g * G::Q0;
#pragma unroll
      for (int q = 0; q < G::Q0; ++q) {
        const float b = brow[q];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = PR::mma(W0[(mt * G::Q0 + q) * kWave + lane], b, acc[mt]);
      }
      const char* p = wsm + G::W0A;
      for (int i = 1; i < H; ++i) {
        const float* WH = reinterpret_cast<const float*>(p);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA);
        f4 nacc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) nacc[mt] = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g);
#pragma unroll
        for (int q = 0; q < 4 * MT; ++q) {
          const float b = activate(acc[q / 4][q % 4], act);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            nacc[mt] = PR::mma(WH[(mt * 4 * MT + q) * kWave + lane], b, nacc[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = nacc[mt];
        p += G::HID;
      }
      const float* WO = reinterpret_cast<const float*>(p) + t * 4 * MT * kWave;
#pragma unroll
      for (int q = 0; q < 4 * MT; ++q) {
        const float b = activate(acc[q / 4][q % 4], act);
        out = PR::mma(WO[q * kWave + lane], b, out);
      }
    }
    const char* p = wsm + G::W0A + (H - 1) * G::HID + G::WOA;
    return out[0] + *reinterpret_cast<const float*>(p);
  } else {
    using VA = typename PR::VA;
    using VT = typename PR::VT;
    f4 out_t = {0.0f, 0.0f, 0.0f, 0.0f};  // K16 part of the output layer
    const VA* W0A = reinterpret_cast<const VA*>(wsm);
    const VT* W0T = reinterpret_cast<const VT*>(wsm + G::W0A);
    for (int t = 0; t < 4; ++t) {
      f4 acc[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      const E* brow = feat + (16 * t + n) * G::ROW;
#pragma unroll
      for (int s = 0; s < G::S0; ++s) {
        const VA b = *reinterpret_cast<const VA*>(brow + 32 * s + 8 * g);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = PR::mma(W0A[(mt * G::S0 + s) * kWave + lane], b, acc[mt]);
      }
      {
        // The K16 tail gets its own accumulator: an MFMA never takes as its
        // accumulator the result of an MFMA of a different shape (that
        // dependency is not reliably interlocked here), the two are summed on
        // the VALU instead.
        const VT b = *reinterpret_cast<const VT*>(brow + G::KMAIN + 4 * g);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] += PR::mmt(W0T[mt * kWave + lane], b, f4{0.0f, 0.0f, 0.0f, 0.0f});
      }
      const char* p = wsm + G::W0A + G::W0T;
      VA bA[G::HS32 > 0 ? G::HS32 : 1];
      VT bT;
      auto pack = [&]() {
#pragma unroll
        for (int s = 0; s < G::HS32; ++s)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            bA[s][j] = to_e<E>(activate(acc[2 * s][j], act));
            bA[s][j + 4] = to_e<E>(activate(acc[2 * s + 1][j], act));
          }
        if constexpr (G::HS16) {
#pragma unroll
          for (int j = 0; j < 4; ++j) bT[j] = to_e<E>(activate(acc[MT - 1][j], act));
        }
      };
      for (int i = 1; i < H; ++i) {
        pack();
        const VA* WA = reinterpret_cast<const VA*>(p);
        const VT* WT = reinterpret_cast<const VT*>(p + G::WHA);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA + G::WHT);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          f4 a = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g);
#pragma unroll
          for (int s = 0; s < G::HS32; ++s) a = PR::mma(WA[(mt * G::HS32 + s) * kWave + lane], bA[s], a);
          if constexpr (G::HS16) a += PR::mmt(WT[mt * kWave + lane], bT, f4{0.0f, 0.0f, 0.0f, 0.0f});
          acc[mt] = a;
        }
        p += G::HID;
      }
      pack();
      const VA* WOA = reinterpret_cast<const VA*>(p) + t * G::HS32 * kWave;
#pragma unroll
      for (int s = 0; s < G::HS32; ++s) out = PR::mma(WOA[s * kWave + lane], bA[s], out);
      if constexpr (G::HS16) {
        const VT* WOT = reinterpret_cast<const VT*>(p + G::WOA) + t * kWave;
        out_t = PR::mmt(WOT[lane], bT, out_t);
      }
    }
    const char* p = wsm + G::W0A + G::W0T + (H - 1) * G::HID + G::WOA + G::WOT;
    return out[0] + out_t[0] + *reinterpret_cast<const float*>(p);
  }
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

struct Ray {
  float o[3], d[3];
  float t0, t1, ds;
  int nseg;
  bool hit;
};

__device__ inline Ray make_ray(const CamDev& cam, int px, int py, int W, int H, const MarchDev& m) {
  Ray r;
  const float nx = (2.0f * px + 1.0f) / (float)W - 1.0f;
  const float ny = 1.0f - (2.0f * py + 1.0f) / (float)H;
  const float sx = cam.aspect * nx;
  if (cam.ortho) {
    const float h = cam.half_extent;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r.o[a] = cam.eye[a] + h * (sx * cam.right[a] + ny * cam.up[a]);
      r.d[a] = cam.fwd[a];
    }
  } else {
    float dd[3], l2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dd[a] = cam.fwd[a] + cam.tan_half * (sx * cam.right[a] + ny * cam.up[a]);
      l2 += dd[a] * dd[a];
    }
    const float inv = 1.0f / sqrtf(l2);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r.o[a] = cam.eye[a];
      r.d[a] = dd[a] * inv;
    }
  }
  float tn = -INFINITY, tf = INFINITY;
  bool miss = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (r.d[a] == 0.0f) {
      if (r.o[a] < -1.0f || r.o[a] > 1.0f) miss = true;
    } else {
      float ta = (-1.0f - r.o[a]) / r.d[a], tb = (1.0f - r.o[a]) / r.d[a];
      if (ta > tb) { float s = ta; ta = tb; tb = s; }
      tn = fmaxf(tn, ta);
      tf = fminf(tf, tb);
    }
  }
  tn = fmaxf(tn, 0.0f);
  r.t0 = tn;
  r.t1 = tf;
  r.hit = !miss && tf > tn;
  if (m.fixed_steps > 0) {
    r.nseg = m.fixed_steps;
    r.ds = (tf - tn) / (float)m.fixed_steps;
  } else {
    r.ds = m.step;
    r.nseg = r.hit ? (int)ceilf((tf - tn) / m.step) : 0;
  }
  if (!r.hit) r.nseg = 0;
  return r;
}

// Segment i of a ray: midpoint parameter and length.
__device__ inline void segment(const Ray& r, int i, bool fixed, float& tm, float& len) {
  const float a0 = r.t0 + (float)i * r.ds;
  float a1 = r.t0 + (float)(i + 1) * r.ds;
  if (!fixed) a1 = fminf(a1, r.t1);
  len = a1 - a0;
  tm = 0.5f * (a0 + a1);
}

// Block -> tile mapping that keeps each XCD (blocks are dealt round-robin to
// the 8 XCDs) on one contiguous range of tiles, so its L2 sees neighbouring
// screen regions.
__device__ inline int xcd_block(int nblocks) {
  const int b = blockIdx.x;
  if (nblocks % 8 != 0) return b;
  const int per = nblocks / 8;
  return (b % 8) * per + b / 8;
}

// ------------------------------------------------------------- kernels

// Waves per workgroup: as many as the LDS holds (weights once, plus one
// input tile per wave), at most kMaxWaves.
constexpr int kMaxWaves = 12;
constexpr int kLdsBytes = 160 * 1024;

template <int P, int C, int F, int L>
int waves_per_block(int H) {
  using G = Geo<P, C, F, L>;
  int w = (kLdsBytes - G::weight_bytes(H)) / G::FEAT_BYTES;
  return w < 1 ? 0 : (w > kMaxWaves ? kMaxWaves : w);
}

template <int P, int C, int F, int L>
__global__ __launch_bounds__(kMaxWaves * 64) void march_kernel(NetDev nd, TFDev tf, ViewBatch vb,
                                                                  MarchDev m, float* out,
                                                                  unsigned long long* stats,
                                                                  int tiles_x, int tiles_y) {
  using G = Geo<P, C, F, L>;
  using E = typename G::E;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  stage_weights<P, C, F, L>(nd, smem);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_per_view = tiles_x * tiles_y;
  const int tile = xcd_block(gridDim.x) * (int)(blockDim.x >> 6) + wave;
  if (tile >= tiles_per_view * vb.n_views) return;
  const int v = tile / tiles_per_view;
  const int tr = tile % tiles_per_view;
  const int px = (tr % tiles_x) * 8 + (lane & 7);
  const int py = (tr / tiles_x) * 8 + (lane >> 3);
  const CamDev& cam = vb.cam[v];
  const bool in_img = px < vb.width && py < vb.height;
  Ray ray = make_ray(cam, in_img ? px : 0, in_img ? py : 0, vb.width, vb.height, m);
  bool active = in_img && ray.hit && ray.nseg > 0;
  const bool fixed = m.fixed_steps > 0;
  E* feat = reinterpret_cast<E*>(smem + G::weight_bytes(nd.H) + wave * G::FEAT_BYTES);
  E* myrow = feat + lane * G::ROW;
  float T = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, A = 0.0f;
  int i = 0;
  const unsigned long long nrays = __builtin_popcountll(__builtin_amdgcn_ballot_w64(active));
  while (__builtin_amdgcn_ballot_w64(active)) {
    float tm, len;
    segment(ray, i, fixed, tm, len);
    if (!active) tm = 0.0f;
    const float sx = ray.o[0] + tm * ray.d[0];
    const float sy = ray.o[1] + tm * ray.d[1];
    const float sz = ray.o[2] + tm * ray.d[2];
    write_features<P, C, F, L>(myrow, nd, cam.key, cam.key_w, active ? sx : 0.0f, active ? sy : 0.0f,
                               active ? sz : 0.0f);
    wave_lds_sync();
    const float logit = mlp_tile<P, C, F, L>(smem, feat, nd.H, nd.act);
    wave_lds_sync();
    if (active) {
      if (len <= 0.0f) {
        active = false;
      } else {
        const float d = sigmoid_f(logit);
        float rgba[4];
        tf_eval(tf, d, rgba);
        const float trn = fast_exp(-rgba[3] * len);
        const float a = 1.0f - trn;
        const float ta = T * a;
        Cr = fmaf(ta, rgba[0], Cr);
        Cg = fmaf(ta, rgba[1], Cg);
        Cb = fmaf(ta, rgba[2], Cb);
        A += ta;
        T *= trn;
        ++i;
        if (T < m.ert_eps || i >= ray.nseg) active = false;
      }
    }
  }
  if (in_img) {
    float4* o = reinterpret_cast<float4*>(out) + ((long long)v * vb.height + py) * vb.width + px;
    *o = make_float4(Cr, Cg, Cb, A);
  }
  if (stats) {
    // samples composited by this wave = sum of per-lane step counts
    unsigned long long mine = (unsigned long long)i;
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
    if (lane == 0) {
      atomicAdd(stats, mine);
      atomicAdd(stats + 1, nrays);
    }
  }
}

template <int P, int C, int F, int L>
__global__ __launch_bounds__(kMaxWaves * 64) void points_kernel(NetDev nd, const float* xyz,
                                                                  long long n, int key, float key_w,
                                                                  float* out) {
  using G = Geo<P, C, F, L>;
  using E = typename G::E;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  stage_weights<P, C, F, L>(nd, smem);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  E* feat = reinterpret_cast<E*>(smem + G::weight_bytes(nd.H) + wave * G::FEAT_BYTES);
  E* myrow = feat + lane * G::ROW;
  const long long nchunks = (n + 63) / 64;
  const int waves = blockDim.x >> 6;
  for (long long c = (long long)blockIdx.x * waves + wave; c < nchunks; c += (long long)gridDim.x * waves) {
    const long long idx = c * 64 + lane;
    const bool ok = idx < n;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    if (ok) {
      x = xyz[3 * idx];
      y = xyz[3 * idx + 1];
      z = xyz[3 * idx + 2];
    }
    write_features<P, C, F, L>(myrow, nd, key, key_w, x, y, z);
    wave_lds_sync();
    const float logit = mlp_tile<P, C, F, L>(smem, feat, nd.H, nd.act);
    wave_lds_sync();
    if (ok) out[idx] = sigmoid_f(logit);
  }
}

// ---------------------------------------------------------- dense DVR

__device__ inline float dense_sample(const float* vol, int nx, int ny, int nz, float px, float py,
                                     float pz) {
  int ix, iy, iz;
  float fx, fy, fz;
  axis_cell(px, nx, ix, fx);
  axis_cell(py, ny, iy, fy);
  axis_cell(pz, nz, iz, fz);
  const long long sy = nx, sz = (long long)nx * ny;
  const float* b = vol + iz * sz + iy * sy + ix;
  const float c00 = b[0] + fx * (b[1] - b[0]);
  const float c10 = b[sy] + fx * (b[sy + 1] - b[sy]);
  const float c01 = b[sz] + fx * (b[sz + 1] - b[sz]);
  const float c11 = b[sz + sy] + fx * (b[sz + sy + 1] - b[sz + sy]);
  const float c0 = c00 + fy * (c10 - c00);
  const float c1 = c01 + fy * (c11 - c01);
  return c0 + fz * (c1 - c0);
}

constexpr int kDenseThreads = 256;

__global__ __launch_bounds__(kDenseThreads) void dense_march_kernel(const float* vol, int nx, int ny,
                                                                    int nz, TFDev tf, ViewBatch vb,
                                                                    MarchDev m, float* out,
                                                                    unsigned long long* stats,
                                                                    int tiles_x, int tiles_y) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_per_view = tiles_x * tiles_y;
  const int tile = xcd_block(gridDim.x) * (kDenseThreads / 64) + wave;
  if (tile >= tiles_per_view * vb.n_views) return;
  const int v = tile / tiles_per_view;
  const int tr = tile % tiles_per_view;
  const int px = (tr % tiles_x) * 8 + (lane & 7);
  const int py = (tr / tiles_x) * 8 + (lane >> 3);
  if (px >= vb.width || py >= vb.height) return;
  const CamDev& cam = vb.cam[v];
  Ray ray = make_ray(cam, px, py, vb.width, vb.height, m);
  const bool fixed = m.fixed_steps > 0;
  float T = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, A = 0.0f;
  int i = 0;
  const float hx = 2.0f / (float)(nx - 1), hy = 2.0f / (float)(ny - 1), hz = 2.0f / (float)(nz - 1);
  for (; i < ray.nseg; ++i) {
    float tm, len;
    segment(ray, i, fixed, tm, len);
    if (len <= 0.0f) break;
    const float sx = ray.o[0] + tm * ray.d[0];
    const float sy = ray.o[1] + tm * ray.d[1];
    const float sz = ray.o[2] + tm * ray.d[2];
    const float d = dense_sample(vol, nx, ny, nz, sx, sy, sz);
    float rgba[4];
    tf_eval(tf, d, rgba);
    if (m.phong) {
      const float gx = (dense_sample(vol, nx, ny, nz, sx + hx, sy, sz) -
                        dense_sample(vol, nx, ny, nz, sx - hx, sy, sz)) / (2.0f * hx);
      const float gy = (dense_sample(vol, nx, ny, nz, sx, sy + hy, sz) -
                        dense_sample(vol, nx, ny, nz, sx, sy - hy, sz)) / (2.0f * hy);
      const float gz = (dense_sample(vol, nx, ny, nz, sx, sy, sz + hz) -
                        dense_sample(vol, nx, ny, nz, sx, sy, sz - hz)) / (2.0f * hz);
      const float gl = sqrtf(gx * gx + gy * gy + gz * gz);
      if (gl >= 1e-6f) {
        const float ndl = fabsf(gx * ray.d[0] + gy * ray.d[1] + gz * ray.d[2]) / gl;
        const float spec = m.ks * powf(ndl, m.shininess);
        const float k = m.ka + m.kd * ndl;
        rgba[0] = rgba[0] * k + spec;
        rgba[1] = rgba[1] * k + spec;
        rgba[2] = rgba[2] * k + spec;
      }
    }
    const float trn = fast_exp(-rgba[3] * len);
    const float ta = T * (1.0f - trn);
    Cr = fmaf(ta, rgba[0], Cr);
    Cg = fmaf(ta, rgba[1], Cg);
    Cb = fmaf(ta, rgba[2], Cb);
    A += ta;
    T *= trn;
    if (T < m.ert_eps) { ++i; break; }
  }
  float4* o = reinterpret_cast<float4*>(out) + ((long long)v * vb.height + py) * vb.width + px;
  *o = make_float4(Cr, Cg, Cb, A);
  if (stats) {
    atomicAdd(stats, (unsigned long long)i);
    if (ray.hit && ray.nseg > 0) atomicAdd(stats + 1, 1ull);
  }
}

__global__ void dense_points_kernel(const float* vol, int nx, int ny, int nz, const float* xyz,
                                    long long n, float* out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = dense_sample(vol, nx, ny, nz, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
}

// --------------------------------------------------------- utilities

__device__ inline void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
  const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
  const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__global__ void sample_points_kernel(uint32_t k0, uint32_t k1, uint32_t c_lo, uint32_t c_hi,
                                     long long n, float* xyz) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)i, (uint32_t)((unsigned long long)i >> 32), c_lo, c_hi};
    uint32_t k[2] = {k0, k1};
    for (int r = 0; r < 10; ++r) {
      if (r > 0) {
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
      }
      philox_round(c, k);
    }
    const float s = 1.0f / 8388608.0f;  // 2^-23
    xyz[3 * i + 0] = -1.0f + (float)(c[0] >> 8) * s;
    xyz[3 * i + 1] = -1.0f + (float)(c[1] >> 8) * s;
    xyz[3 * i + 2] = -1.0f + (float)(c[2] >> 8) * s;
  }
}

__global__ void cast_f16_kernel(const float* src, _Float16* dst, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (_Float16)src[i];
}

__global__ void cast_bf16_kernel(const float* src, __bf16* dst, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (__bf16)src[i];
}

thread_local char g_hip_err[256];

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(g_hip_err, sizeof(g_hip_err), "%s", hipGetErrorString(e));
    return 2;
  }
  return 0;
}

int grid_blocks(long long work, int per_block, int cap) {
  long long b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

template <int P, int C, int F, int L>
int launch_render_t(const NetDev& nd, const TFDev& tf, const ViewBatch& vb, const MarchDev& m, float* out,
                    unsigned long long* stats, hipStream_t st) {
  using G = Geo<P, C, F, L>;
  const int tx = (vb.width + 7) / 8, ty = (vb.height + 7) / 8;
  const long long tiles = (long long)tx * ty * vb.n_views;
  const int wpb = waves_per_block<P, C, F, L>(nd.H);
  if (wpb < 1) return 1;
  long long blocks = (tiles + wpb - 1) / wpb;
  if (blocks % 8) blocks += 8 - blocks % 8;
  const size_t shm = (size_t)G::weight_bytes(nd.H) + (size_t)wpb * G::FEAT_BYTES;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)march_kernel<P, C, F, L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    attr = true;
  }
  hipLaunchKernelGGL((march_kernel<P, C, F, L>), dim3((unsigned)blocks), dim3(wpb * 64), shm, st,
                     nd, tf, vb, m, out, stats, tx, ty);
  return check_launch();
}

template <int P, int C, int F, int L>
int launch_points_t(const NetDev& nd, const float* xyz, long long n, int key, float key_w, float* out,
                    hipStream_t st) {
  using G = Geo<P, C, F, L>;
  const int wpb = waves_per_block<P, C, F, L>(nd.H);
  if (wpb < 1) return 1;
  const size_t shm = (size_t)G::weight_bytes(nd.H) + (size_t)wpb * G::FEAT_BYTES;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)points_kernel<P, C, F, L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kLdsBytes);
    attr = true;
  }
  // each block walks several 64-point chunks per wave so the weight staging is amortised
  const int blocks = grid_blocks((n + 63) / 64, wpb * 8, device_cus() * 4);
  hipLaunchKernelGGL((points_kernel<P, C, F, L>), dim3(blocks), dim3(wpb * 64), shm, st, nd, xyz,
                     n, key, key_w, out);
  return check_launch();
}

// Dispatch over the compiled configurations.
template <template <int, int, int, int> class Fn, typename... Args>
int dispatch(int prec, int C, int F, int L, Args&&... args) {
#define FV_CASE(P_, C_, F_, L_) \
  if (prec == P_ && C == C_ && F == F_ && L == L_) return Fn<P_, C_, F_, L_>::run(args...);
#define FV_CASES(P_)         \
  FV_CASE(P_, 32, 8, 4)      \
  FV_CASE(P_, 32, 16, 8)     \
  FV_CASE(P_, 48, 8, 4)      \
  FV_CASE(P_, 48, 16, 8)
  FV_CASES(kF32)
  FV_CASES(kF16)
  FV_CASES(kBF16)
#undef FV_CASES
#undef FV_CASE
  return 1;
}

template <int P, int C, int F, int L>
struct RenderFn {
  static int run(const NetDev& nd, const TFDev& tf, const ViewBatch& vb, const MarchDev& m, float* out,
                 unsigned long long* stats, hipStream_t st) {
    return launch_render_t<P, C, F, L>(nd, tf, vb, m, out, stats, st);
  }
};

template <int P, int C, int F, int L>
struct PointsFn {
  static int run(const NetDev& nd, const float* xyz, long long n, int key, float key_w, float* out,
                 hipStream_t st) {
    return launch_points_t<P, C, F, L>(nd, xyz, n, key, key_w, out, st);
  }
};

}  // namespace

// ---------------------------------------------------------- launchers

const char* last_hip_error() { return g_hip_err; }

int launch_render(const NetDev& net, int prec, const TFDev& tf, const ViewBatch& views, const MarchDev& m,
                  float* out, unsigned long long* stats, void* stream) {
  if (m.phong) return 1;  // forward-mode gradient render: not compiled in this build
  return dispatch<RenderFn>(prec, net.C, net.F, net.L, net, tf, views, m, out, stats, (hipStream_t)stream);
}

int launch_points(const NetDev& net, int prec, const float* xyz, long long n, int key, float key_w,
                  float* out_d, float* out_g, void* stream) {
  if (out_g) return 1;  // forward-mode gradient: not compiled in this build
  return dispatch<PointsFn>(prec, net.C, net.F, net.L, net, xyz, n, key, key_w, out_d, (hipStream_t)stream);
}

int launch_render_dense(const float* vol, int nx, int ny, int nz, const TFDev& tf, const ViewBatch& vb,
                        const MarchDev& m, float* out, unsigned long long* stats, void* stream) {
  const int tx = (vb.width + 7) / 8, ty = (vb.height + 7) / 8;
  const long long tiles = (long long)tx * ty * vb.n_views;
  long long blocks = (tiles + 3) / 4;
  if (blocks % 8) blocks += 8 - blocks % 8;
  hipLaunchKernelGGL(dense_march_kernel, dim3((unsigned)blocks), dim3(kDenseThreads), 0, (hipStream_t)stream,
                     vol, nx, ny, nz, tf, vb, m, out, stats, tx, ty);
  return check_launch();
}

int launch_dense_points(const float* vol, int nx, int ny, int nz, const float* xyz, long long n, float* out,
                        void* stream) {
  const int blocks = grid_blocks(n, 256, device_cus() * 16);
  hipLaunchKernelGGL(dense_points_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, vol, nx, ny, nz,
                     xyz, n, out);
  return check_launch();
}

int launch_sample_points(uint64_t seed, uint64_t counter, long long n, float* xyz, void* stream) {
  const int blocks = grid_blocks(n, 256, device_cus() * 16);
  hipLaunchKernelGGL(sample_points_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (uint32_t)seed,
                     (uint32_t)(seed >> 32), (uint32_t)counter, (uint32_t)(counter >> 32), n, xyz);
  return check_launch();
}

int launch_cast(const float* src, void* dst, long long count, int dst_dtype, void* stream) {
  const int blocks = grid_blocks(count, 256, device_cus() * 16);
  if (dst_dtype == kF16)
    hipLaunchKernelGGL(cast_f16_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, src,
                       (_Float16*)dst, count);
  else
    hipLaunchKernelGGL(cast_bf16_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, src, (__bf16*)dst,
                       count);
  return check_launch();
}

size_t train_workspace_bytes(const NetDev&, long long) { return 0; }

int launch_train(const NetDev&, float*, float*, float*, float*, const float*, long long, const float*,
                 const float*, int, float, float, float, float, float, int, float*, float*, float*, float*,
                 float*, void*, size_t, void*) {
  return 1;
}

}  // namespace fvsrn_detail
