// The fused network evaluation shared by the render and point kernels:
// weight staging into MFMA fragment order, the per-lane network input, and
// the MLP over a wave's 64 input rows. Two modes:
//  * value mode: each lane owns one sample (row = lane);
//  * gradient mode (forward-mode differentiation, Sec. 6): the four lanes of
//    a quad own one sample; lane 4s + q holds column q of sample s, where
//    q = 0 is the value and q = 1..3 the tangent d/dx, d/dy, d/dz. Tangent
//    columns go through the same matrices (no bias), and each activation
//    multiplies them by the derivative of the activation at the value
//    column's pre-activation, fetched from the quad's first lane with DPP.
#pragma once
#include "fvsrn_common.hpp"

namespace fvsrn_detail {

// GK selects the latent gather of an FP16 network: 0 generic (FP32
// accumulation, grid type chosen at run time), 1 FP16 grid and 2 uint8 grid,
// both accumulated in packed FP16 (one gather path per instantiation keeps
// the register peak down). A BF16 network on an FP16 grid (GK 1) also sums
// the corners in packed FP16 and rounds the sums to BF16 for its row (FP16
// keeps three more bits than the row). G16 says that a packed path is used.
// TE: time encoding of the input (0 latent only, 1 direct, 2 Fourier, 3 both).
// FM: the Fourier features come from a general matrix (random Fourier
// features) instead of the octave construction.
template <int P_, int C_, int F_, int L_, int ACT_, int GK_ = 0, int TE_ = 0, int FM_ = 0>
struct Cfg {
  static constexpr int P = P_, C = C_, F = F_, L = L_, ACT = ACT_;
  static constexpr int GK = GK_;
  static constexpr int TE = TE_;
  static constexpr bool FM = FM_ != 0;
  static constexpr bool G16 = GK_ != 0;
  using G = Geo<P, C, F, L, TE>;
  using E = typename G::E;
};

// Per-lane constants of the lane's column.
struct LaneRole {
  bool is_val;   // value column (always true in value mode)
  int axis;      // tangent axis 0..2 (gradient mode, !is_val)
  float qmask;   // 1 for the value column: biases apply to it only
  float toff;    // 0 (value) or 1/4 revolution: sin(x + pi/2) = cos(x)
  float tmul;    // 0 (value) or 2 pi
  float tadd;    // 1 (value) or 0
};

__device__ inline LaneRole value_role() { return LaneRole{true, 0, 1.0f, 0.0f, 0.0f, 1.0f}; }

__device__ inline LaneRole grad_role(int q) {
  LaneRole r;
  r.is_val = q == 0;
  r.axis = q > 0 ? q - 1 : 0;
  r.qmask = q == 0 ? 1.0f : 0.0f;
  r.toff = q == 0 ? 0.0f : 0.25f;
  r.tmul = q == 0 ? 0.0f : k2Pi;
  r.tadd = q == 0 ? 1.0f : 0.0f;
  return r;
}

// ------------------------------------------------------ weight staging

// The packed uint8 gather hands the row its weighted code sums times this
// power of two (see latent_column_q).
constexpr float kCodeSumScale = 1.0f / 1024.0f;

// Converts the FP32 master weights into A fragments in LDS (lane order), with
// the first layer's columns permuted to the input-row order and each hidden
// layer's columns permuted so that the previous layer's D fragments are this
// layer's B fragments. Layers 0..H-1 are scaled by 1/(2 pi) for the periodic
// activations (their accumulators then hold revolutions).
template <class CF>
__device__ void stage_weights(const NetDev& nd, char* smem) {
  using G = typename CF::G;
  using E = typename CF::E;
  constexpr int C = CF::C, F = CF::F, L = CF::L, MT = G::MT;
  constexpr int K0 = G::K0IN;
  const int H = nd.H, NO = nd.NO;
  const float* w = nd.weights;
  const float sc = CF::ACT == kIdentity ? 1.0f : kInv2Pi;
  // a single uint8 keyframe on the packed path: the de-quantisation is folded
  // into layer 0 (latent columns times the channel scale, the channel offsets
  // into the bias), so the input row carries the weighted code sums (times
  // kCodeSumScale, which the latent columns undo)
  const bool fold = CF::GK == 2 && nd.grid_u8 && nd.K == 1;
  const float* dq = nd.dequant;
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long off_b0 = (long long)C * K0;
  auto off_layer = [&](int i) -> long long {  // W_i for 1 <= i <= H
    return (long long)C * K0 + C + (long long)(i - 1) * (C * C + C);
  };
  // FP16/BF16 networks receive 2 cos(.) in the Fourier cosine block (see
  // write_features); their cosine columns carry half the weight.
  auto w0 = [&](int o, int col) -> float {
    if (col < G::KF) {
      const float half = (CF::P != kF32 && col >= F + 3 * L) ? 0.5f : 1.0f;
      const float qs = (fold && col < F) ? dq[2 * col + 1] * (1.0f / kCodeSumScale) : 1.0f;
      return w[(long long)o * K0 + 3 + col] * qs * sc * half;
    }
    if (col < G::KMAIN) return 0.0f;
    const int t = col - G::KMAIN;
    if (t < 3) return w[(long long)o * K0 + t] * sc;
    if (t == 3) {
      float b = w[off_b0 + o];
      if (fold)
        for (int ch = 0; ch < F; ++ch) b = fmaf(w[(long long)o * K0 + 3 + ch], dq[2 * ch], b);
      return b * sc;
    }
    if (t < 4 + G::TIN) return w[(long long)o * K0 + 3 + G::KF + (t - 4)] * sc;  // time inputs
    return 0.0f;
  };
  char* p = smem;
  if constexpr (CF::P == kF32) {
    float* W0 = reinterpret_cast<float*>(p);
    for (int e = tid; e < MT * G::Q0 * kWave; e += nt) {
      const int lane = e % kWave, q = (e / kWave) % G::Q0, mt = e / (kWave * G::Q0);
      W0[e] = w0(16 * mt + (lane & 15), (lane >> 4) * G::Q0 + q);
    }
    p += G::W0A;
    for (int i = 1; i < H; ++i) {
      const float* Wi = w + off_layer(i);
      float* WH = reinterpret_cast<float*>(p);
      for (int e = tid; e < MT * 4 * MT * kWave; e += nt) {
        const int lane = e % kWave, q = (e / kWave) % (4 * MT), mt = e / (kWave * 4 * MT);
        const int ch = 16 * (q / 4) + 4 * (lane >> 4) + (q % 4);
        WH[e] = Wi[(16 * mt + (lane & 15)) * C + ch] * sc;
      }
      float* BHp = reinterpret_cast<float*>(p + G::WHA);
      for (int e = tid; e < C; e += nt) BHp[e] = Wi[C * C + e] * sc;
      p += G::HID;
    }
    const float* Wo = w + off_layer(H);
    float* WO = reinterpret_cast<float*>(p);
    for (int e = tid; e < 4 * 4 * MT * kWave; e += nt) {
      const int lane = e % kWave, q = (e / kWave) % (4 * MT), t = e / (kWave * 4 * MT);
      const int ch = 16 * (q / 4) + 4 * (lane >> 4) + (q % 4);
      const int o = (lane & 15) - 4 * t;  // output o of N-tile t sits in row 4t + o
      WO[e] = (o >= 0 && o < NO) ? Wo[o * C + ch] : 0.0f;
    }
    p += G::WOA;
    if (tid < 4) reinterpret_cast<float*>(p)[tid] = tid < NO ? Wo[NO * C + tid] : 0.0f;
  } else {
    E* W0A = reinterpret_cast<E*>(p);
    for (int e = tid; e < MT * G::S0 * kWave * 8; e += nt) {
      const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::S0, mt = (e >> 9) / G::S0;
      W0A[e] = to_e<E>(w0(16 * mt + (lane & 15), 32 * s + 8 * (lane >> 4) + j));
    }
    // tail step: K32 fragments over [x y z 1 0 0 0 0] (w0 is zero past column KMAIN + 3)
    E* W0T = reinterpret_cast<E*>(p + G::W0A);
    for (int e = tid; e < MT * kWave * 8; e += nt) {
      const int j = e & 7, lane = (e >> 3) & 63, mt = e >> 9;
      W0T[e] = to_e<E>(w0(16 * mt + (lane & 15), G::KMAIN + 8 * (lane >> 4) + j));
    }
    p += G::W0A + G::W0T;
    for (int i = 1; i < H; ++i) {
      const float* Wi = w + off_layer(i);
      E* WA = reinterpret_cast<E*>(p);
      for (int e = tid; e < MT * G::HS32 * kWave * 8; e += nt) {
        const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::HS32, mt = (e >> 9) / G::HS32;
        const int g = lane >> 4;
        const int ch = j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4);
        WA[e] = to_e<E>(Wi[(16 * mt + (lane & 15)) * C + ch] * sc);
      }
      if constexpr (G::HS16) {
        E* WT = reinterpret_cast<E*>(p + G::WHA);
        for (int e = tid; e < MT * kWave * 4; e += nt) {
          const int j = e & 3, lane = (e >> 2) & 63, mt = e >> 8;
          const int ch = 16 * (MT - 1) + 4 * (lane >> 4) + j;
          WT[e] = to_e<E>(Wi[(16 * mt + (lane & 15)) * C + ch] * sc);
        }
      }
      float* BHp = reinterpret_cast<float*>(p + G::WHA + G::WHT);
      for (int e = tid; e < C; e += nt) BHp[e] = Wi[C * C + e] * sc;
      p += G::HID;
    }
    const float* Wo = w + off_layer(H);
    E* WOA = reinterpret_cast<E*>(p);
    for (int e = tid; e < 4 * G::HS32 * kWave * 8; e += nt) {
      const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::HS32, t = (e >> 9) / G::HS32;
      const int g = lane >> 4;
      const int ch = j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4);
      const int o = (lane & 15) - 4 * t;  // output o of N-tile t sits in row 4t + o
      WOA[e] = to_e<E>((o >= 0 && o < NO) ? Wo[o * C + ch] : 0.0f);
    }
    if constexpr (G::HS16) {
      E* WOT = reinterpret_cast<E*>(p + G::WOA);
      for (int e = tid; e < 4 * kWave * 4; e += nt) {
        const int j = e & 3, lane = (e >> 2) & 63, t = e >> 8;
        const int ch = 16 * (MT - 1) + 4 * (lane >> 4) + j;
        const int o = (lane & 15) - 4 * t;
        WOT[e] = to_e<E>((o >= 0 && o < NO) ? Wo[o * C + ch] : 0.0f);
      }
    }
    p += G::WOA + G::WOT;
    if (tid < 4) reinterpret_cast<float*>(p)[tid] = tid < NO ? Wo[NO * C + tid] : 0.0f;
  }
}

// ------------------------------------------------------ network input

// Latent source: one or two keyframe grids and their blend weights (Sec. 8).
struct LatentSrc {
  const void* g0;
  const void* g1;  // == nullptr: single keyframe
  float w0, w1;
  int R;
  int dtype;              // storage: kF32, kF16 or kU8
  unsigned bytes;         // one keyframe grid (< 2^31, checked by the host)
  const float* dq0;       // uint8 grids: (offset, scale) per channel of each keyframe
  const float* dq1;
};

// Buffer resource over one keyframe grid. The corner fetches then address
// the grid as (per-lane cell offset) + (wave-uniform corner offset, held in
// an SGPR) + (immediate for the second 16 bytes), so a sample's eight corners
// cost no per-lane address arithmetic beyond the cell offset.
__device__ inline __amdgpu_buffer_rsrc_t grid_rsrc(const void* g, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(g), 0, (int)bytes, 0x00020000);
}

__device__ inline uint4 load16(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

__device__ inline uint2 load8(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// The F uint8 codes of one vertex as F/4 dwords (F = 8 or 16).
template <int F>
__device__ inline void load_codes(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, unsigned d[F / 4]) {
  if constexpr (F == 16) {
    const uint4 q = load16(r, voff, soff);
    d[0] = q.x;
    d[1] = q.y;
    d[2] = q.z;
    d[3] = q.w;
  } else {
    static_assert(F == 8, "uint8 grids: F = 8 or 16");
    const uint2 q = load8(r, voff, soff);
    d[0] = q.x;
    d[1] = q.y;
  }
}

__device__ inline LatentSrc make_latent_src(const NetDev& nd, int key, float key_w) {
  LatentSrc s;
  const size_t esz = nd.grid_u8 ? 1 : (nd.grid_f16 ? 2 : 4);
  const char* base = reinterpret_cast<const char*>(nd.latent);
  s.g0 = base + (size_t)key * (size_t)nd.key_stride * esz;
  s.g1 = nd.K > 1 ? base + (size_t)(key + 1) * (size_t)nd.key_stride * esz : nullptr;
  s.w0 = nd.K > 1 ? 1.0f - key_w : 1.0f;
  s.w1 = key_w;
  s.R = nd.R;
  s.dtype = nd.grid_u8 ? kU8 : (nd.grid_f16 ? kF16 : kF32);
  s.bytes = (unsigned)((size_t)nd.key_stride * esz);
  s.dq0 = nd.grid_u8 ? nd.dequant + (size_t)key * nd.F * 2 : nullptr;
  s.dq1 = (nd.grid_u8 && nd.K > 1) ? s.dq0 + nd.F * 2 : nullptr;
  return s;
}

// Corner offsets of a cell in elements: x fastest, then y, then z.
__device__ inline void corner_offsets(unsigned sx, unsigned sy, unsigned sz, unsigned off[8]) {
  off[0] = 0;
  off[1] = sx;
  off[2] = sy;
  off[3] = sx + sy;
  off[4] = sz;
  off[5] = sz + sx;
  off[6] = sz + sy;
  off[7] = sz + sx + sy;
}

// z += w * G[corner][0..F) for the 8 corners of the cell at offset `base`.
// A uint8 grid adds sum_c w_c (offset + scale * code_c) per channel, i.e. the
// de-quantised vertex values (Sec. 4.2), as scale * (sum_c w_c code_c) +
// offset * (sum_c w_c).
template <int F>
__device__ inline void gather8(const void* grid, int dtype, unsigned bytes, unsigned base, unsigned sx, unsigned sy,
                               unsigned sz, const float w[8], float* z, const float* dq) {
  unsigned off[8];
  corner_offsets(sx, sy, sz, off);
  const __amdgpu_buffer_rsrc_t r = grid_rsrc(grid, bytes);
  if (dtype == kU8) {
    float acc[F], wsum = 0.0f;
#pragma unroll
    for (int j = 0; j < F; ++j) acc[j] = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      unsigned d[F / 4];
      load_codes<F>(r, base, off[c], d);
#pragma unroll
      for (int q = 0; q < F / 4; ++q) {
        acc[4 * q + 0] = fmaf(w[c], (float)((d[q] >> 0) & 0xffu), acc[4 * q + 0]);
        acc[4 * q + 1] = fmaf(w[c], (float)((d[q] >> 8) & 0xffu), acc[4 * q + 1]);
        acc[4 * q + 2] = fmaf(w[c], (float)((d[q] >> 16) & 0xffu), acc[4 * q + 2]);
        acc[4 * q + 3] = fmaf(w[c], (float)((d[q] >> 24) & 0xffu), acc[4 * q + 3]);
      }
      wsum += w[c];
    }
#pragma unroll
    for (int j = 0; j < F; ++j) z[j] += fmaf(dq[2 * j + 1], acc[j], dq[2 * j] * wsum);
  } else if (dtype == kF16) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
#pragma unroll
      for (int q = 0; q < F / 8; ++q) {
        const h8 hv = __builtin_bit_cast(h8, load16(r, base * 2u + 16u * q, off[c] * 2u));
#pragma unroll
        for (int j = 0; j < 8; ++j) z[8 * q + j] = fmaf(w[c], (float)hv[j], z[8 * q + j]);
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
#pragma unroll
      for (int q = 0; q < F / 4; ++q) {
        const float4 v = __builtin_bit_cast(float4, load16(r, base * 4u + 16u * q, off[c] * 4u));
        z[4 * q + 0] = fmaf(w[c], v.x, z[4 * q + 0]);
        z[4 * q + 1] = fmaf(w[c], v.y, z[4 * q + 1]);
        z[4 * q + 2] = fmaf(w[c], v.z, z[4 * q + 2]);
        z[4 * q + 3] = fmaf(w[c], v.w, z[4 * q + 3]);
      }
    }
  }
}

// Trilinear latent vector (value lanes) or its derivative along the lane's
// axis (tangent lanes), blended over the keyframes, added into z[0..F).
template <int F>
__device__ inline void latent_column(const LatentSrc& ls, const LaneRole& role, float px, float py, float pz,
                                     float* z) {
  int ix, iy, iz;
  float fx, fy, fz, dx, dy, dz;
  axis_cell(px, ls.R, ix, fx, dx);
  axis_cell(py, ls.R, iy, fy, dy);
  axis_cell(pz, ls.R, iz, fz, dz);
  // per-axis factors of the low / high corner: value (1-f, f); along the
  // differentiated axis (-df/dp, df/dp)
  const bool tx = !role.is_val && role.axis == 0, ty = !role.is_val && role.axis == 1,
             tz = !role.is_val && role.axis == 2;
  const float x0 = tx ? -dx : 1.0f - fx, x1 = tx ? dx : fx;
  const float y0 = ty ? -dy : 1.0f - fy, y1 = ty ? dy : fy;
  const float z0 = tz ? -dz : 1.0f - fz, z1 = tz ? dz : fz;
  const unsigned R = (unsigned)ls.R;
  const unsigned sx = F, sy = R * F, sz = R * R * F;
  const unsigned base = (unsigned)iz * sz + (unsigned)iy * sy + (unsigned)ix * sx;
  float w[8] = {x0 * y0 * z0, x1 * y0 * z0, x0 * y1 * z0, x1 * y1 * z0,
                x0 * y0 * z1, x1 * y0 * z1, x0 * y1 * z1, x1 * y1 * z1};
  float wa[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) wa[c] = w[c] * ls.w0;
  gather8<F>(ls.g0, ls.dtype, ls.bytes, base, sx, sy, sz, wa, z, ls.dq0);
  if (ls.g1) {
#pragma unroll
    for (int c = 0; c < 8; ++c) wa[c] = w[c] * ls.w1;
    gather8<F>(ls.g1, ls.dtype, ls.bytes, base, sx, sy, sz, wa, z, ls.dq1);
  }
}

// FP16 variant of latent_column for an FP16 grid feeding an FP16 network:
// the eight corner products are accumulated pairwise in packed FP16 (each
// corner is one v_pk_fma per two channels) and land in the input row without
// a conversion. The row is rounded to FP16 for the MFMA in any case.
// Two phases, so that work independent of the grid can be placed while the
// corner loads are in flight: begin() finds the cell, its weights and issues
// the first keyframe's corner loads; finish() accumulates them and gathers a
// second keyframe, if any.
template <int F>
struct LatentColumnH {
  h8 raw[8][F / 8];  // the first keyframe's corners, as loaded
  float xy[4], z0, z1;
  unsigned base, off[8];

  __device__ inline void begin(const LatentSrc& ls, const LaneRole& role, float px, float py, float pz) {
    int ix, iy, iz;
    float fx, fy, fz, dx, dy, dz;
    axis_cell_h(px, ls.R, ix, fx, dx);
    axis_cell_h(py, ls.R, iy, fy, dy);
    axis_cell_h(pz, ls.R, iz, fz, dz);
    const bool tx = !role.is_val && role.axis == 0, ty = !role.is_val && role.axis == 1,
               tz = !role.is_val && role.axis == 2;
    const float x0 = tx ? -dx : 1.0f - fx, x1 = tx ? dx : fx;
    const float y0 = ty ? -dy : 1.0f - fy, y1 = ty ? dy : fy;
    z0 = tz ? -dz : 1.0f - fz;
    z1 = tz ? dz : fz;
    const unsigned R = (unsigned)ls.R;
    const unsigned sx = F, sy = R * F, sz = R * R * F;
    base = vertex_offset(ix, iy, iz, sx, sy, sz);
    corner_offsets(sx, sy, sz, off);
    xy[0] = x0 * y0;
    xy[1] = x1 * y0;
    xy[2] = x0 * y1;
    xy[3] = x1 * y1;
    load(ls.g0, ls.bytes);
  }

  __device__ inline void load(const void* g, unsigned bytes) {
    const __amdgpu_buffer_rsrc_t r = grid_rsrc(g, bytes);
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
      for (int q = 0; q < F / 8; ++q) raw[c][q] = __builtin_bit_cast(h8, load16(r, base * 2u + 16u * q, off[c] * 2u));
  }

  // z2 += sum over corners of weight * corner, weights x * y * (z * kw) in
  // FP32, rounded once to FP16 in pairs (x0, x1): the FMAs broadcast either half
  __device__ inline void accumulate(float kw, h2* z2) const {
    const float zk[2] = {z0 * kw, z1 * kw};
    h2 wp[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      wp[j] = __builtin_convertvector((f2{xy[2 * (j & 1)] * zk[j >> 1], xy[2 * (j & 1) + 1] * zk[j >> 1]}), h2);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const _Float16 wh = wp[c >> 1][c & 1];
      const h2 w2 = {wh, wh};
#pragma unroll
      for (int q = 0; q < F / 8; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const h2 v2 = {raw[c][q][2 * j], raw[c][q][2 * j + 1]};
          z2[4 * q + j] = w2 * v2 + z2[4 * q + j];
        }
    }
  }

  __device__ inline void finish(const LatentSrc& ls, h2* z2) {
#pragma unroll
    for (int j = 0; j < F / 2; ++j) z2[j] = h2{(_Float16)0.0f, (_Float16)0.0f};
    accumulate(ls.w0, z2);  // w0 = 1 for a single keyframe
    if (ls.g1) {
      load(ls.g1, ls.bytes);
      accumulate(ls.w1, z2);
    }
  }
};

// The same gather in one phase: each corner's loads are consumed as they
// arrive (the render, whose 8x8 ray tiles mostly hit in L1, keeps 4 waves per
// SIMD with it).
template <int F>
__device__ inline void latent_column_h(const LatentSrc& ls, const LaneRole& role, float px, float py, float pz,
                                       h2* z2) {
  int ix, iy, iz;
  float fx, fy, fz, dx, dy, dz;
  axis_cell_h(px, ls.R, ix, fx, dx);
  axis_cell_h(py, ls.R, iy, fy, dy);
  axis_cell_h(pz, ls.R, iz, fz, dz);
  const bool tx = !role.is_val && role.axis == 0, ty = !role.is_val && role.axis == 1,
             tz = !role.is_val && role.axis == 2;
  const float x0 = tx ? -dx : 1.0f - fx, x1 = tx ? dx : fx;
  const float y0 = ty ? -dy : 1.0f - fy, y1 = ty ? dy : fy;
  const float z0 = tz ? -dz : 1.0f - fz, z1 = tz ? dz : fz;
  const unsigned R = (unsigned)ls.R;
  const unsigned sx = F, sy = R * F, sz = R * R * F;
  const unsigned base = vertex_offset(ix, iy, iz, sx, sy, sz);
  unsigned off[8];
  corner_offsets(sx, sy, sz, off);
  const float xy[4] = {x0 * y0, x1 * y0, x0 * y1, x1 * y1};
#pragma unroll
  for (int j = 0; j < F / 2; ++j) z2[j] = h2{(_Float16)0.0f, (_Float16)0.0f};
#pragma unroll
  for (int key = 0; key < 2; ++key) {
    const void* g = key == 0 ? ls.g0 : ls.g1;
    if (key == 1 && !g) break;
    const __amdgpu_buffer_rsrc_t r = grid_rsrc(g, ls.bytes);
    const float kw = key == 0 ? ls.w0 : ls.w1;  // 1 for a single keyframe
    const float zk[2] = {z0 * kw, z1 * kw};
    h2 wp[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      wp[j] = __builtin_convertvector((f2{xy[2 * (j & 1)] * zk[j >> 1], xy[2 * (j & 1) + 1] * zk[j >> 1]}), h2);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const _Float16 wh = wp[c >> 1][c & 1];
      const h2 w2 = {wh, wh};
#pragma unroll
      for (int q = 0; q < F / 8; ++q) {
        const h8 hv = __builtin_bit_cast(h8, load16(r, base * 2u + 16u * q, off[c] * 2u));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const h2 v2 = {hv[2 * j], hv[2 * j + 1]};
          z2[4 * q + j] = w2 * v2 + z2[4 * q + j];
        }
      }
    }
  }
}

// uint8 variant of LatentColumnH (Sec. 4.2's quantised grid) for an FP16
// network. A byte permute next to a zero byte turns each code pair into two
// FP16 subnormals code * 2^-24 (exact: the FP16 denormals are kept), and the
// corner weights carry 2^14, so each packed FMA adds w * code * 2^-10 with
// one rounding, as w * code would be: the row receives the weighted code sums
// times 2^-10 (kCodeSumScale), and no per-corner subtraction is needed.
// Tangent lanes (forward mode, weights up to (R - 1) / 2) carry 2^7 instead
// and scale their sums by 2^7 at the end. The sums keep 1/8 of a code at the
// top of the range. With one keyframe they go to the row as they are (layer 0
// holds the de-quantisation, times 2^10); with two they are de-quantised and
// blended.
template <int F>
__device__ inline void latent_column_q(const LatentSrc& ls, const LaneRole& role, float px, float py, float pz,
                                       h2* z2) {
  int ix, iy, iz;
  float fx, fy, fz, dx, dy, dz;
  axis_cell(px, ls.R, ix, fx, dx);
  axis_cell(py, ls.R, iy, fy, dy);
  axis_cell(pz, ls.R, iz, fz, dz);
  const bool tx = !role.is_val && role.axis == 0, ty = !role.is_val && role.axis == 1,
             tz = !role.is_val && role.axis == 2;
  const float x0 = tx ? -dx : 1.0f - fx, x1 = tx ? dx : fx;
  const float y0 = ty ? -dy : 1.0f - fy, y1 = ty ? dy : fy;
  const float z0 = tz ? -dz : 1.0f - fz, z1 = tz ? dz : fz;
  const unsigned R = (unsigned)ls.R;
  const unsigned sx = F, sy = R * F, sz = R * R * F;
  const unsigned base = (unsigned)iz * sz + (unsigned)iy * sy + (unsigned)ix * sx;
  unsigned off[8];
  corner_offsets(sx, sy, sz, off);
  const float w[8] = {x0 * y0 * z0, x1 * y0 * z0, x0 * y1 * z0, x1 * y1 * z0,
                      x0 * y0 * z1, x1 * y0 * z1, x0 * y1 * z1, x1 * y1 * z1};
  const float wscale = role.is_val ? 16384.0f : 128.0f;
  float zf[F];
#pragma unroll
  for (int j = 0; j < F; ++j) zf[j] = 0.0f;
#pragma unroll
  for (int key = 0; key < 2; ++key) {
    const void* g = key == 0 ? ls.g0 : ls.g1;
    if (key == 1 && !g) break;
    const __amdgpu_buffer_rsrc_t r = grid_rsrc(g, ls.bytes);
    const float kw = ls.g1 != nullptr ? (key == 0 ? ls.w0 : ls.w1) : 1.0f;
    const float* dq = key == 0 ? ls.dq0 : ls.dq1;
    h2 acc[F / 2];
#pragma unroll
    for (int j = 0; j < F / 2; ++j) acc[j] = h2{(_Float16)0.0f, (_Float16)0.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const _Float16 wh = (_Float16)(w[c] * wscale);
      const h2 w2 = {wh, wh};
      unsigned d[F / 4];
      load_codes<F>(r, base, off[c], d);
#pragma unroll
      for (int q = 0; q < F / 4; ++q) {
        const h2 lo = __builtin_bit_cast(h2, __builtin_amdgcn_perm(0u, d[q], 0x04010400u));
        const h2 hi = __builtin_bit_cast(h2, __builtin_amdgcn_perm(0u, d[q], 0x04030402u));
        acc[2 * q] = w2 * lo + acc[2 * q];
        acc[2 * q + 1] = w2 * hi + acc[2 * q + 1];
      }
    }
    if (!role.is_val) {
      const h2 up = {(_Float16)128.0f, (_Float16)128.0f};
#pragma unroll
      for (int j = 0; j < F / 2; ++j) acc[j] *= up;
    }
    if (!ls.g1) {
      // one keyframe: layer 0 holds the de-quantisation (see stage_weights)
#pragma unroll
      for (int j = 0; j < F / 2; ++j) z2[j] = acc[j];
      return;
    }
    // de-quantise: offset * sum(w) + scale * sum(w code), blended over keyframes
    const float wsum = ((w[0] + w[1]) + (w[2] + w[3])) + ((w[4] + w[5]) + (w[6] + w[7]));
#pragma unroll
    for (int j = 0; j < F / 2; ++j) {
      const float a0 = (float)acc[j][0] * (1.0f / kCodeSumScale), a1 = (float)acc[j][1] * (1.0f / kCodeSumScale);
      zf[2 * j] = fmaf(kw, fmaf(dq[4 * j + 1], a0, dq[4 * j] * wsum), zf[2 * j]);
      zf[2 * j + 1] = fmaf(kw, fmaf(dq[4 * j + 3], a1, dq[4 * j + 2] * wsum), zf[2 * j + 1]);
    }
  }
#pragma unroll
  for (int j = 0; j < F / 2; ++j) z2[j] = h2{(_Float16)zf[2 * j], (_Float16)zf[2 * j + 1]};
}

// Time inputs (Sec. 8) of the normalised time tau, in the row's tail order:
// tau (direct), then sin and cos of pi 2^k tau for k < 4 (Fourier).
template <int TE>
__device__ inline void time_features(float tau, float* tf) {
  int j = 0;
  if constexpr (TE == 1 || TE == 3) tf[j++] = tau;
  if constexpr (TE >= 2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      tf[j + k] = sin_rev(0.5f * (float)(1 << k) * tau);
      tf[j + 4 + k] = cos_rev(0.5f * (float)(1 << k) * tau);
    }
  }
}

// Normalised time: [lo, hi] onto [-1, 1], clamped (scale = 2 / (hi - lo)).
__device__ inline float time_tau(float t, float lo, float hi, float scale) {
  return fmaf(__builtin_amdgcn_fmed3f(t, lo, hi) - lo, scale, -1.0f);
}

// Builds this lane's input row at position p and writes it to `row` (LDS).
// tf: the sample's time inputs (Geo::TIN values; ignored without a time
// encoding); they do not depend on p, so tangent rows get zeros there.
// OVERLAP (FP16 network on an FP16 grid): issue the corner loads, build the
// Fourier features, then accumulate the corners, so that the features hide
// the loads' latency; it holds the loaded corners in registers meanwhile
// (worth it at 3 waves per SIMD, where the random point gathers wait on L2;
// the render's 8x8 ray tiles hit in L1 and run at 4 waves without it).
template <class CF, bool GRAD, bool OVERLAP = false>
__device__ inline void write_features(typename CF::E* row, const LatentSrc& ls, const LaneRole& role, float px,
                                      float py, float pz, const float* tf = nullptr,
                                      const float (*fm)[3] = nullptr) {
  using G = typename CF::G;
  using E = typename CF::E;
  constexpr int F = CF::F, L = CF::L;
  float v[G::KROW];
#pragma unroll
  for (int j = 0; j < G::KROW; ++j) v[j] = 0.0f;
  constexpr bool packed_latent = CF::G16 && (CF::P == kF16 || (CF::P == kBF16 && CF::GK == 1));
  h2 zh[F / 2];
  LatentColumnH<F> lch;
  if constexpr (packed_latent && CF::GK == 2) {
    latent_column_q<F>(ls, role, px, py, pz, zh);
  } else if constexpr (packed_latent && OVERLAP) {
    lch.begin(ls, role, px, py, pz);
    // keep the Fourier features below between the loads and their use
    __builtin_amdgcn_sched_barrier(0);
  } else if constexpr (packed_latent) {
    latent_column_h<F>(ls, role, px, py, pz, zh);
  } else {
    latent_column<F>(ls, role, px, py, pz, v);
  }
  // Fourier features sin/cos(pi 2^k p_a). FP32 network: each octave from the
  // exact power-of-two phase 2^(k-1) p_a (revolutions). FP16/BF16 networks:
  // octave 0 directly, the others by the double-angle identities written for
  // g = 2 cos x: sin 2x = sin x * g, g(2x) = g^2 - 2 -- one multiply and one
  // FMA per octave (error ~2^k * 1e-7, far below the FP16 rounding of the
  // row). The row then holds 2 cos in the cosine block; the staged weights of
  // those columns are halved.
  const float pp[3] = {px, py, pz};
  float mv = 1.0f, ma[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (GRAD) {
    mv = role.is_val ? 1.0f : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) ma[a] = (!role.is_val && role.axis == a) ? 1.0f : 0.0f;
  }
  constexpr float cs = CF::P == kF32 ? 1.0f : 2.0f;  // scale of the cosine block
  float sd[3], gd[3];
  if constexpr (CF::P != kF32 && !CF::FM) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sd[a] = sin_rev(0.5f * pp[a]);
      gd[a] = 2.0f * cos_rev(0.5f * pp[a]);
    }
  }
  if constexpr (CF::FM) {
    // a general Fourier matrix (rows in revolutions per world unit): phase
    // r_j = row_j . p, features sin / cs cos(2 pi r_j); tangent along axis a:
    // 2 pi row_ja cos, -2 pi row_ja sin
#pragma unroll
    for (int j = 0; j < 3 * L; ++j) {
      const float r = fmaf(fm[j][0], px, fmaf(fm[j][1], py, fm[j][2] * pz));
      const float s = sin_rev(r), c = cs * cos_rev(r);
      if constexpr (GRAD) {
        const float wm = k2Pi * (ma[0] * fm[j][0] + ma[1] * fm[j][1] + ma[2] * fm[j][2]);
        v[F + j] = fmaf(c, wm * (1.0f / cs), s * mv);
        v[F + 3 * L + j] = fmaf(-s, wm * cs, c * mv);
      } else {
        v[F + j] = s;
        v[F + 3 * L + j] = c;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < (CF::FM ? 0 : L); ++k) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float s, c;  // sin and cs * cos of the octave's phase
      if constexpr (CF::P == kF32) {
        const float ph = pp[a] * (float)(1 << k) * 0.5f;
        s = sin_rev(ph);
        c = cos_rev(ph);
      } else {
        s = sd[a];
        c = gd[a];
        if (k + 1 < L) {
          sd[a] = s * c;
          gd[a] = fmaf(c, c, -2.0f);
          // keep the value itself for the row: otherwise the compiler redoes
          // the FMA inside a one-value mixed-precision conversion instead of
          // converting pairs
          asm("" : "+v"(gd[a]));
        }
      }
      if constexpr (GRAD) {
        // d/dp_a sin(w p_a) = w cos(w p_a), d/dp_a cos(w p_a) = -w sin(w p_a)
        const float wm = kPi * (float)(1 << k) * ma[a];
        v[F + 3 * k + a] = fmaf(c, wm * (1.0f / cs), s * mv);
        v[F + 3 * L + 3 * k + a] = fmaf(-s, wm * cs, c * mv);
      } else {
        v[F + 3 * k + a] = s;
        v[F + 3 * L + 3 * k + a] = c;
      }
    }
    // forward mode: keep each octave's work together, which lowers the
    // register peak of the feature build
    if constexpr (GRAD) __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (packed_latent && CF::GK == 1 && OVERLAP) {
    __builtin_amdgcn_sched_barrier(0);
    lch.finish(ls, zh);
  }
  if constexpr (GRAD) {
    v[G::KMAIN + 0] = role.is_val ? px : (role.axis == 0 ? 1.0f : 0.0f);
    v[G::KMAIN + 1] = role.is_val ? py : (role.axis == 1 ? 1.0f : 0.0f);
    v[G::KMAIN + 2] = role.is_val ? pz : (role.axis == 2 ? 1.0f : 0.0f);
    v[G::KMAIN + 3] = role.qmask;
  } else {
    v[G::KMAIN + 0] = px;
    v[G::KMAIN + 1] = py;
    v[G::KMAIN + 2] = pz;
    v[G::KMAIN + 3] = 1.0f;
  }
#pragma unroll
  for (int j = 0; j < G::TIN; ++j) v[G::KMAIN + 4 + j] = (GRAD && !role.is_val) ? 0.0f : tf[j];
  if constexpr (CF::P == kF32) {
    float4* dst = reinterpret_cast<float4*>(row);
#pragma unroll
    for (int q = 0; q < G::KROW / 4; ++q) dst[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
    using V8 = typename PrecT<CF::P>::VA;
    V8* dst = reinterpret_cast<V8*>(row);
#pragma unroll
    for (int q = 0; q < G::KROW / 8; ++q) {
      V8 x;
      bool done = false;
      if constexpr (packed_latent) {
        if (q < F / 8) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if constexpr (CF::P == kF16) {
              x[2 * j] = zh[4 * q + j][0];
              x[2 * j + 1] = zh[4 * q + j][1];
            } else {
              x[2 * j] = to_e<E>((float)zh[4 * q + j][0]);
              x[2 * j + 1] = to_e<E>((float)zh[4 * q + j][1]);
            }
          }
          done = true;
        }
      }
      if (!done) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = to_e<E>(v[8 * q + j]);
      }
      dst[q] = x;
    }
  }
}

// ---------------------------------------------------------- activation

// Activation of one accumulator element r (pre-activation in revolutions
// for the periodic activations). Gradient mode: value lanes return the
// activation of their pre-activation, tangent lanes the activation's
// derivative at the value column's pre-activation times their own tangent.
template <int ACT, bool GRAD>
__device__ inline float act_el(float r, const LaneRole& role) {
  if constexpr (!GRAD) {
    if constexpr (ACT == kSine) {
      return sin_rev(r);
    } else if constexpr (ACT == kSnakeAlt) {  // 0.5 x + sin^2 x with x = 2 pi r
      const float s = sin_rev(r);
      return fmaf(kPi, r, s * s);
    } else {
      return r;
    }
  } else {
    const float rv = quad_bcast0(r);
    if constexpr (ACT == kSine) {
      // value: sin(2 pi rv); tangent: cos(2 pi rv) * 2 pi r
      return sin_rev(rv + role.toff) * fmaf(r, role.tmul, role.tadd);
    } else if constexpr (ACT == kSnakeAlt) {
      const float s = sin_rev(rv);
      const float val = fmaf(kPi, rv, s * s);
      const float tan = (0.5f + sin_rev(2.0f * rv)) * k2Pi * r;
      return role.is_val ? val : tan;
    } else {
      return r;
    }
  }
}

// ------------------------------------------------------------- the MLP

// Runs the network on the wave's 64 input rows and returns the output-layer
// pre-activation of this lane's own row (logit of its sample, or the
// logit's derivative for tangent lanes). Pairs of N-tiles are processed
// together so that two independent MFMA / activation chains interleave.
template <class CF, bool GRAD>
__device__ inline f4 mlp_tile(const char* wsm, const typename CF::E* feat, int H, const LaneRole& role) {
  using G = typename CF::G;
  using PR = PrecT<CF::P>;
  using E = typename CF::E;
  constexpr int MT = G::MT;
  constexpr int NT = 2;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15;
  if constexpr (CF::P == kF32) {
    f4 out[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) out[u] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const float* W0 = reinterpret_cast<const float*>(wsm);
    for (int tp = 0; tp < 4; tp += NT) {
      f4 acc[NT][MT];
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[u][mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < G::Q0; ++q) {
        float b[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) b[u] = feat[(16 * (tp + u) + n) * G::ROW + g * G::Q0 + q];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float a = W0[(mt * G::Q0 + q) * kWave + lane];
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[u][mt] = PR::mma(a, b[u], acc[u][mt]);
        }
      }
      const char* p = wsm + G::W0A;
      for (int i = 1; i < H; ++i) {
        const float* WH = reinterpret_cast<const float*>(p);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA);
        f4 nacc[NT][MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const f4 bias = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g) * role.qmask;
#pragma unroll
          for (int u = 0; u < NT; ++u) nacc[u][mt] = bias;
        }
#pragma unroll
        for (int q = 0; q < 4 * MT; ++q) {
          float b[NT];
#pragma unroll
          for (int u = 0; u < NT; ++u) b[u] = act_el<CF::ACT, GRAD>(acc[u][q / 4][q % 4], role);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const float a = WH[(mt * 4 * MT + q) * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) nacc[u][mt] = PR::mma(a, b[u], nacc[u][mt]);
          }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[u][mt] = nacc[u][mt];
        p += G::HID;
      }
      const float* WO = reinterpret_cast<const float*>(p);
#pragma unroll
      for (int q = 0; q < 4 * MT; ++q) {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const float b = act_el<CF::ACT, GRAD>(acc[u][q / 4][q % 4], role);
          out[u] = PR::mma(WO[((tp + u) * 4 * MT + q) * kWave + lane], b, out[u]);
        }
      }
    }
    const f4 bo = *reinterpret_cast<const f4*>(wsm + G::W0A + (H - 1) * G::HID + G::WOA);
    return out[0] + out[1] + bo * role.qmask;
  } else {
    using VA = typename PR::VA;
    using VT = typename PR::VT;
    const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f4 out[NT], out_t[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) out[u] = out_t[u] = zero;
    const VA* W0A = reinterpret_cast<const VA*>(wsm);
    const VA* W0T = reinterpret_cast<const VA*>(wsm + G::W0A);
    for (int tp = 0; tp < 4; tp += NT) {
      f4 acc[NT][MT];
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[u][mt] = zero;
#pragma unroll
      for (int s = 0; s < G::S0; ++s) {
        VA b[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u)
          b[u] = *reinterpret_cast<const VA*>(feat + (16 * (tp + u) + n) * G::ROW + 32 * s + 8 * g);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const VA a = W0A[(mt * G::S0 + s) * kWave + lane];
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[u][mt] = PR::mma(a, b[u], acc[u][mt]);
        }
      }
      {
        // Tail step [x y z 1 (time) 0 ...] as one more K32 step on the same
        // accumulators (lanes past the tail's 8 or 16 columns read them again;
        // their A slots are zero). Keeping one MFMA shape per accumulator matters: a
        // 16x16x32 result used as the accumulator of the next 16x16x16 MFMA
        // is not reliably interlocked.
        VA b[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u)
          b[u] = *reinterpret_cast<const VA*>(feat + (16 * (tp + u) + n) * G::ROW + G::KMAIN + 8 * (g % (G::KT / 8)));
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const VA a = W0T[mt * kWave + lane];
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[u][mt] = PR::mma(a, b[u], acc[u][mt]);
        }
      }
      const char* p = wsm + G::W0A + G::W0T;
      VA bA[NT][G::HS32 > 0 ? G::HS32 : 1];
      VT bT[NT];
      auto pack = [&]() {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
#pragma unroll
          for (int s = 0; s < G::HS32; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              bA[u][s][j] = to_e<E>(act_el<CF::ACT, GRAD>(acc[u][2 * s][j], role));
              bA[u][s][j + 4] = to_e<E>(act_el<CF::ACT, GRAD>(acc[u][2 * s + 1][j], role));
            }
          if constexpr (G::HS16) {
#pragma unroll
            for (int j = 0; j < 4; ++j) bT[u][j] = to_e<E>(act_el<CF::ACT, GRAD>(acc[u][MT - 1][j], role));
          }
        }
      };
      for (int i = 1; i < H; ++i) {
        pack();
        const VA* WA = reinterpret_cast<const VA*>(p);
        const VT* WT = reinterpret_cast<const VT*>(p + G::WHA);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA + G::WHT);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const f4 bias = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g) * role.qmask;
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[u][mt] = bias;
#pragma unroll
          for (int s = 0; s < G::HS32; ++s) {
            const VA a = WA[(mt * G::HS32 + s) * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[u][mt] = PR::mma(a, bA[u][s], acc[u][mt]);
          }
          if constexpr (G::HS16) {
            const VT a = WT[mt * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[u][mt] += PR::mmt(a, bT[u], zero);
          }
        }
        p += G::HID;
      }
      pack();
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const VA* WOA = reinterpret_cast<const VA*>(p) + (tp + u) * G::HS32 * kWave;
#pragma unroll
        for (int s = 0; s < G::HS32; ++s) out[u] = PR::mma(WOA[s * kWave + lane], bA[u][s], out[u]);
        if constexpr (G::HS16) {
          const VT* WOT = reinterpret_cast<const VT*>(p + G::WOA) + (tp + u) * kWave;
          out_t[u] = PR::mmt(WOT[lane], bT[u], out_t[u]);
        }
      }
    }
    const f4 bo = *reinterpret_cast<const f4*>(wsm + G::W0A + G::W0T + (H - 1) * G::HID + G::WOA + G::WOT);
    f4 y = out[0] + out[1] + bo * role.qmask;
    if constexpr (G::HS16) y += out_t[0] + out_t[1];
    return y;
  }
}

}  // namespace fvsrn_detail
