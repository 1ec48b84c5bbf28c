// Adjoint (reverse-mode) density gradient of the value-mode tile (Sec. 6:
// backpropagation through the network to the sample position). For each
// pair of N-tiles the forward pass keeps every activated layer's derivative
// in registers; the output weights, scaled by the last derivative, are then
// pulled back through the transposed layers on MFMA down to dy/d(input row),
// which replaces the pair's input rows in LDS. Each lane finally contracts
// its own row with the input row's Jacobian: identity for x, y, z, the
// Fourier derivatives, and the derivatives of the trilinear weights for the
// latent columns.
#pragma once
#include "fvsrn_net.hpp"

namespace fvsrn_detail {

// d act / d x at the pre-activation r (revolutions for the periodic
// activations, x = 2 pi r).
template <int ACT>
__device__ inline float act_deriv(float r) {
  if constexpr (ACT == kSine) return cos_rev(r);
  else if constexpr (ACT == kSnakeAlt) return 0.5f + sin_rev(2.0f * r);
  else return 1.0f;
}

// Transposed fragments at p (Geo::back_bytes(H) bytes): W_i^T of the hidden
// layers in the A-operand order of their forward counterparts (rows: input
// channels; K slots: output channels in the D-fragment order), W_0^T with one
// row per input-row column, then the output weights in FP32. Unscaled: in x
// units the chain rule reads dy/dh_i = W_i^T (dy/dh_{i+1} * act'(x_i)), and
// the cosine columns take their true weights (the pass differentiates with
// respect to the true cos features).
template <class CF>
__device__ void stage_backward_adj(const NetDev& nd, char* p) {
  using G = typename CF::G;
  using E = typename CF::E;
  constexpr int C = CF::C, F = CF::F, L = CF::L, MT = G::MT, MB0 = G::MB0;
  const int H = nd.H, K0 = G::K0IN;
  const float* w = nd.weights;
  const int tid = threadIdx.x, nt = blockDim.x;
  auto off_layer = [&](int i) -> long long {  // W_i for 1 <= i <= H
    return (long long)C * K0 + C + (long long)(i - 1) * (C * C + C);
  };
  auto w0t = [&](int o, int col) -> float {  // layer 0 weight of input-row column col
    if (col < G::KF) return w[(long long)o * K0 + 3 + col];
    if (col >= G::KMAIN && col < G::KMAIN + 3) return w[(long long)o * K0 + (col - G::KMAIN)];
    return 0.0f;
  };
  if constexpr (CF::P == kF32) {
    for (int i = 1; i < H; ++i) {
      const float* Wi = w + off_layer(i);
      float* WB = reinterpret_cast<float*>(p);
      for (int e = tid; e < MT * 4 * MT * kWave; e += nt) {
        const int lane = e % kWave, q = (e / kWave) % (4 * MT), mt = e / (kWave * 4 * MT);
        const int ch = 16 * (q / 4) + 4 * (lane >> 4) + (q % 4);
        WB[e] = Wi[(long long)ch * C + 16 * mt + (lane & 15)];
      }
      p += G::WBH;
    }
    float* WB0 = reinterpret_cast<float*>(p);
    for (int e = tid; e < MB0 * 4 * MT * kWave; e += nt) {
      const int lane = e % kWave, q = (e / kWave) % (4 * MT), m = e / (kWave * 4 * MT);
      const int ch = 16 * (q / 4) + 4 * (lane >> 4) + (q % 4);
      WB0[e] = w0t(ch, 16 * m + (lane & 15));
    }
    p += G::WB0;
  } else {
    for (int i = 1; i < H; ++i) {
      const float* Wi = w + off_layer(i);
      E* WA = reinterpret_cast<E*>(p);
      for (int e = tid; e < MT * G::HS32 * kWave * 8; e += nt) {
        const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::HS32, mt = (e >> 9) / G::HS32;
        const int g = lane >> 4;
        const int ch = j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4);
        WA[e] = to_e<E>(Wi[(long long)ch * C + 16 * mt + (lane & 15)]);
      }
      if constexpr (G::HS16) {
        E* WT = reinterpret_cast<E*>(p + G::WHA);
        for (int e = tid; e < MT * kWave * 4; e += nt) {
          const int j = e & 3, lane = (e >> 2) & 63, mt = e >> 8;
          const int ch = 16 * (MT - 1) + 4 * (lane >> 4) + j;
          WT[e] = to_e<E>(Wi[(long long)ch * C + 16 * mt + (lane & 15)]);
        }
      }
      p += G::WBH;
    }
    E* W0A = reinterpret_cast<E*>(p);
    for (int e = tid; e < MB0 * G::HS32 * kWave * 8; e += nt) {
      const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::HS32, m = (e >> 9) / G::HS32;
      const int g = lane >> 4;
      const int ch = j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4);
      W0A[e] = to_e<E>(w0t(ch, 16 * m + (lane & 15)));
    }
    if constexpr (G::HS16) {
      E* W0T = reinterpret_cast<E*>(p + G::WB0A);
      for (int e = tid; e < MB0 * kWave * 4; e += nt) {
        const int j = e & 3, lane = (e >> 2) & 63, m = e >> 8;
        const int ch = 16 * (MT - 1) + 4 * (lane >> 4) + j;
        W0T[e] = to_e<E>(w0t(ch, 16 * m + (lane & 15)));
      }
    }
    p += G::WB0;
  }
  float* WO = reinterpret_cast<float*>(p);
  const float* Wo = w + off_layer(H);
  for (int e = tid; e < C; e += nt) WO[e] = Wo[e];  // output 0: the density logit
}

// Layers whose activation derivatives the first forward pass of the adjoint
// keeps in registers. A deeper network's first H - kAdjKeep layers are run a
// second time, from the input rows, once the backward pass has reached them.
constexpr int kAdjKeep = 4;

// Forward and adjoint pass of the wave's 64 input rows through a network of
// HH activated layers (wsm: forward fragments, bsm: stage_backward_adj). On
// return the 64 rows of `feat` hold dy/d(input row) in the input-row column
// order (y: output 0, the logit), and the lane's own logit is returned.
// With HH > kAdjKeep the first pass keeps the derivatives of the last
// kAdjKeep layers only; after the backward pass through them, a second
// forward pass over the first S = HH - kAdjKeep layers supplies theirs.
template <class CF, int HH>
__device__ __attribute__((always_inline)) inline float mlp_tile_adj(const char* wsm, const char* bsm,
                                                                  typename CF::E* feat) {
  using G = typename CF::G;
  using PR = PrecT<CF::P>;
  using E = typename CF::E;
  // N-tiles per pass: two interleaved chains, one for the FP32 c = 48
  // network (whose saved derivatives would not fit the registers twice)
  constexpr int MT = G::MT, MB0 = G::MB0, NT = (CF::P == kF32 && CF::C == 48) ? 1 : 2, ACT = CF::ACT;
  constexpr int S = HH > kAdjKeep ? HH - kAdjKeep : 0, HD = HH - S;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15;
  const LaneRole role = value_role();
  const float* wout = reinterpret_cast<const float*>(bsm + (HH - 1) * G::WBH + G::WB0);
  const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  f4 out[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) out[u] = zero;
  if constexpr (CF::P == kF32) {
    f4 wo[MT];  // output weights in the D-fragment order: channel 16 mt + 4 g + j
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) wo[mt] = *reinterpret_cast<const f4*>(wout + 16 * mt + 4 * g);
    const float* W0 = reinterpret_cast<const float*>(wsm);
    for (int tp = 0; tp < 4; tp += NT) {
      f4 acc[NT][MT];
      // layer 0 pre-activations of the pair's input rows
      auto layer0 = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[u][mt] = zero;
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
      };
      // pre-activations of the hidden layer at p from the activations hb
      auto hidden = [&](const char* p, const f4 (&hb)[NT][MT]) __attribute__((always_inline)) {
        const float* WH = reinterpret_cast<const float*>(p);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const f4 bias = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g);
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[u][mt] = bias;
        }
#pragma unroll
        for (int q = 0; q < 4 * MT; ++q)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const float a = WH[(mt * 4 * MT + q) * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[u][mt] = PR::mma(a, hb[u][q / 4][q % 4], acc[u][mt]);
          }
      };
      f4 e[NT][MT];
      // e <- (W_i^T e) * act'(x_{i-1})
      auto back = [&](int i, const f4 (&d)[NT][MT]) __attribute__((always_inline)) {
        const float* WB = reinterpret_cast<const float*>(bsm + (i - 1) * G::WBH);
        f4 nu[NT][MT];
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) nu[u][mt] = zero;
#pragma unroll
        for (int q = 0; q < 4 * MT; ++q)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const float a = WB[(mt * 4 * MT + q) * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) nu[u][mt] = PR::mma(a, e[u][q / 4][q % 4], nu[u][mt]);
          }
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) e[u][mt] = nu[u][mt] * d[u][mt];
      };
      layer0();
      // forward, keeping act' of the last HD activated layers
      f4 der[HD][NT][MT];
      const char* p = wsm + G::W0A;
#pragma unroll
      for (int i = 0; i < HH; ++i) {
        f4 hb[NT][MT];
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float r = acc[u][mt][j];
              hb[u][mt][j] = act_el<ACT, false>(r, role);
              if (i >= S) der[i - S][u][mt][j] = act_deriv<ACT>(r);
            }
        if (i + 1 < HH) {
          hidden(p, hb);
          p += G::HID;
        } else {
          const float* WO = reinterpret_cast<const float*>(p);
#pragma unroll
          for (int q = 0; q < 4 * MT; ++q)
#pragma unroll
            for (int u = 0; u < NT; ++u)
              out[u] = PR::mma(WO[((tp + u) * 4 * MT + q) * kWave + lane], hb[u][q / 4][q % 4], out[u]);
        }
      }
      // backward: e_i = dy/dh_{i+1} * act'(x_i), dy/dh_i = W_i^T e_i
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) e[u][mt] = wo[mt] * der[HD - 1][u][mt];
#pragma unroll
      for (int i = HH - 1; i > S; --i) back(i, der[i - 1 - S]);
      if constexpr (S > 0) {
        // second forward pass over the first S layers for their act'; the
        // memory clobber makes it reload its operands, so the compiler
        // cannot keep the first pass's values alive to reuse them
        asm volatile("" ::: "memory");
        f4 der0[S][NT][MT];
        layer0();
        const char* p0 = wsm + G::W0A;
#pragma unroll
        for (int i = 0; i < S; ++i) {
          f4 hb[NT][MT];
#pragma unroll
          for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const float r = acc[u][mt][j];
                der0[i][u][mt][j] = act_deriv<ACT>(r);
                hb[u][mt][j] = i + 1 < S ? act_el<ACT, false>(r, role) : 0.0f;
              }
          if (i + 1 < S) {
            hidden(p0, hb);
            p0 += G::HID;
          }
        }
#pragma unroll
        for (int i = S; i >= 1; --i) back(i, der0[i - 1]);
      }
      // dy/d(input row) = W_0^T e_0, written over the pair's rows
      const float* WB0 = reinterpret_cast<const float*>(bsm + (HH - 1) * G::WBH);
#pragma unroll
      for (int m = 0; m < MB0; ++m) {
        f4 u0[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) u0[u] = zero;
#pragma unroll
        for (int q = 0; q < 4 * MT; ++q) {
          const float a = WB0[(m * 4 * MT + q) * kWave + lane];
#pragma unroll
          for (int u = 0; u < NT; ++u) u0[u] = PR::mma(a, e[u][q / 4][q % 4], u0[u]);
        }
        if (16 * m + 4 * g < G::KROW) {
#pragma unroll
          for (int u = 0; u < NT; ++u)
            *reinterpret_cast<f4*>(feat + (16 * (tp + u) + n) * G::ROW + 16 * m + 4 * g) = u0[u];
        }
      }
    }
    const f4 bo = *reinterpret_cast<const f4*>(wsm + G::W0A + (HH - 1) * G::HID + G::WOA);
    float y = bo[0];
#pragma unroll
    for (int u = 0; u < NT; ++u) y += out[u][0];
    return y;
  } else {
    using VA = typename PR::VA;
    using VT = typename PR::VT;
    constexpr int HS32 = G::HS32;
    // output weights in the packed B-operand order of the last hidden layer
    VA woA[HS32];
    VT woT;
#pragma unroll
    for (int s = 0; s < HS32; ++s)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        woA[s][j] = to_e<E>(wout[j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4)]);
#pragma unroll
    for (int j = 0; j < 4; ++j) woT[j] = to_e<E>(G::HS16 ? wout[16 * (MT - 1) + 4 * g + j] : 0.0f);
    f4 out_t[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) out_t[u] = zero;
    const VA* W0A = reinterpret_cast<const VA*>(wsm);
    const VA* W0T = reinterpret_cast<const VA*>(wsm + G::W0A);
    for (int tp = 0; tp < 4; tp += NT) {
      f4 acc[NT][MT];
      // layer 0 pre-activations of the pair's input rows
      auto layer0 = [&]() __attribute__((always_inline)) {
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
      };
      // pre-activations of the hidden layer at p from the activations bA, bT
      auto hidden = [&](const char* p, const VA (&bA)[NT][HS32], const VT (&bT)[NT]) __attribute__((always_inline)) {
        const VA* WA = reinterpret_cast<const VA*>(p);
        const VT* WT = reinterpret_cast<const VT*>(p + G::WHA);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA + G::WHT);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const f4 bias = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g);
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[u][mt] = bias;
#pragma unroll
          for (int s = 0; s < HS32; ++s) {
            const VA a = WA[(mt * HS32 + s) * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[u][mt] = PR::mma(a, bA[u][s], acc[u][mt]);
          }
          if constexpr (G::HS16) {
            const VT a = WT[mt * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[u][mt] += PR::mmt(a, bT[u], zero);
          }
        }
      };
      // activations (packed B order) and, with d set, act' of acc
      auto activate = [&](VA (&bA)[NT][HS32], VT (&bT)[NT], VA* dA, VT* dT, bool want_h)
          __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
#pragma unroll
          for (int s = 0; s < HS32; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float r0 = acc[u][2 * s][j], r1 = acc[u][2 * s + 1][j];
              if (want_h) {
                bA[u][s][j] = to_e<E>(act_el<ACT, false>(r0, role));
                bA[u][s][j + 4] = to_e<E>(act_el<ACT, false>(r1, role));
              }
              if (dA) {
                dA[u * HS32 + s][j] = to_e<E>(act_deriv<ACT>(r0));
                dA[u * HS32 + s][j + 4] = to_e<E>(act_deriv<ACT>(r1));
              }
            }
          if constexpr (G::HS16) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float r = acc[u][MT - 1][j];
              if (want_h) bT[u][j] = to_e<E>(act_el<ACT, false>(r, role));
              if (dT) dT[u][j] = to_e<E>(act_deriv<ACT>(r));
            }
          }
        }
      };
      VA eA[NT][HS32];
      VT eT[NT];
      // e <- (W_i^T e) * act'(x_{i-1})
      auto back = [&](int i, const VA (&dA)[NT][HS32], const VT (&dT)[NT]) __attribute__((always_inline)) {
        const VA* WBA = reinterpret_cast<const VA*>(bsm + (i - 1) * G::WBH);
        const VT* WBT = reinterpret_cast<const VT*>(bsm + (i - 1) * G::WBH + G::WHA);
        f4 nu[NT][MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
          for (int u = 0; u < NT; ++u) nu[u][mt] = zero;
#pragma unroll
          for (int s = 0; s < HS32; ++s) {
            const VA a = WBA[(mt * HS32 + s) * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) nu[u][mt] = PR::mma(a, eA[u][s], nu[u][mt]);
          }
          if constexpr (G::HS16) {
            const VT a = WBT[mt * kWave + lane];
#pragma unroll
            for (int u = 0; u < NT; ++u) nu[u][mt] += PR::mmt(a, eT[u], zero);
          }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
#pragma unroll
          for (int s = 0; s < HS32; ++s) {
            VA x;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              x[j] = to_e<E>(nu[u][2 * s][j]);
              x[j + 4] = to_e<E>(nu[u][2 * s + 1][j]);
            }
            eA[u][s] = x * dA[u][s];
          }
          if constexpr (G::HS16) {
            VT x;
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = to_e<E>(nu[u][MT - 1][j]);
            eT[u] = x * dT[u];
          }
        }
      };
      layer0();
      // forward, keeping act' of the last HD activated layers in the packed B order
      VA dA[HD][NT][HS32];
      VT dT[HD][NT];
      VA bA[NT][HS32];
      VT bT[NT];
      const char* p = wsm + G::W0A + G::W0T;
#pragma unroll
      for (int i = 0; i < HH; ++i) {
        if (i >= S) activate(bA, bT, &dA[i - S][0][0], dT[i - S], true);
        else activate(bA, bT, nullptr, nullptr, true);
        if (i + 1 < HH) {
          hidden(p, bA, bT);
          p += G::HID;
        } else {
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            const VA* WOA = reinterpret_cast<const VA*>(p) + (tp + u) * HS32 * kWave;
#pragma unroll
            for (int s = 0; s < HS32; ++s) out[u] = PR::mma(WOA[s * kWave + lane], bA[u][s], out[u]);
            if constexpr (G::HS16) {
              const VT* WOT = reinterpret_cast<const VT*>(p + G::WOA) + (tp + u) * kWave;
              out_t[u] = PR::mmt(WOT[lane], bT[u], out_t[u]);
            }
          }
        }
      }
      // backward in the packed B order: e_i = dy/dh_{i+1} * act'(x_i)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
#pragma unroll
        for (int s = 0; s < HS32; ++s) eA[u][s] = woA[s] * dA[HD - 1][u][s];
        if constexpr (G::HS16) eT[u] = woT * dT[HD - 1][u];
      }
#pragma unroll
      for (int i = HH - 1; i > S; --i) back(i, dA[i - 1 - S], dT[i - 1 - S]);
      if constexpr (S > 0) {
        // second forward pass over the first S layers for their act'; the
        // memory clobber makes it reload its operands, so the compiler
        // cannot keep the first pass's values alive to reuse them
        asm volatile("" ::: "memory");
        VA dA0[S][NT][HS32];
        VT dT0[S][NT];
        layer0();
        const char* p0 = wsm + G::W0A + G::W0T;
#pragma unroll
        for (int i = 0; i < S; ++i) {
          activate(bA, bT, &dA0[i][0][0], dT0[i], i + 1 < S);
          if (i + 1 < S) {
            hidden(p0, bA, bT);
            p0 += G::HID;
          }
        }
#pragma unroll
        for (int i = S; i >= 1; --i) back(i, dA0[i - 1], dT0[i - 1]);
      }
      // dy/d(input row) = W_0^T e_0, written over the pair's rows
      const VA* WB0A = reinterpret_cast<const VA*>(bsm + (HH - 1) * G::WBH);
      const VT* WB0T = reinterpret_cast<const VT*>(bsm + (HH - 1) * G::WBH + G::WB0A);
#pragma unroll
      for (int m = 0; m < MB0; ++m) {
        f4 u0[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) u0[u] = zero;
#pragma unroll
        for (int s = 0; s < HS32; ++s) {
          const VA a = WB0A[(m * HS32 + s) * kWave + lane];
#pragma unroll
          for (int u = 0; u < NT; ++u) u0[u] = PR::mma(a, eA[u][s], u0[u]);
        }
        if constexpr (G::HS16) {
          const VT a = WB0T[m * kWave + lane];
#pragma unroll
          for (int u = 0; u < NT; ++u) u0[u] += PR::mmt(a, eT[u], zero);
        }
        if (16 * m + 4 * g < G::KROW) {
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            VT x;
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = to_e<E>(u0[u][j]);
            *reinterpret_cast<VT*>(feat + (16 * (tp + u) + n) * G::ROW + 16 * m + 4 * g) = x;
          }
        }
      }
    }
    const f4 bo = *reinterpret_cast<const f4*>(wsm + G::W0A + G::W0T + (HH - 1) * G::HID + G::WOA + G::WOT);
    float y = out[0][0] + out[1][0] + bo[0];
    if constexpr (G::HS16) y += out_t[0][0] + out_t[1][0];
    return y;
  }
}

// g += sum_f u_f d z_f / d p: the latent columns' share of the gradient. The
// trilinear weights are differentiated per axis (d frac / d p is zero outside
// the domain) and each corner's vector is contracted with u first (one dot
// product per corner and keyframe). A uint8 grid's per-channel offset drops
// out: the derivatives of the eight weights sum to zero.
template <int F>
__device__ inline void latent_vjp(const LatentSrc& ls, float px, float py, float pz, const float* u, float g[3]) {
  int ix, iy, iz;
  float fx, fy, fz, dx, dy, dz;
  axis_cell(px, ls.R, ix, fx, dx);
  axis_cell(py, ls.R, iy, fy, dy);
  axis_cell(pz, ls.R, iz, fz, dz);
  const float X[2] = {1.0f - fx, fx}, Y[2] = {1.0f - fy, fy}, Z[2] = {1.0f - fz, fz};
  const float DX[2] = {-dx, dx}, DY[2] = {-dy, dy}, DZ[2] = {-dz, dz};
  const unsigned R = (unsigned)ls.R;
  const unsigned sx = F, sy = R * F, sz = R * R * F;
  const unsigned base = (unsigned)iz * sz + (unsigned)iy * sy + (unsigned)ix * sx;
  unsigned off[8];
  corner_offsets(sx, sy, sz, off);
#pragma unroll
  for (int key = 0; key < 2; ++key) {
    const void* grid = key == 0 ? ls.g0 : ls.g1;
    if (key == 1 && !grid) break;
    const float kw = key == 0 ? ls.w0 : ls.w1;
    const float* dq = key == 0 ? ls.dq0 : ls.dq1;
    const __amdgpu_buffer_rsrc_t r = grid_rsrc(grid, ls.bytes);
    float us[F];
#pragma unroll
    for (int f = 0; f < F; ++f) us[f] = ls.dtype == kU8 ? u[f] * dq[2 * f + 1] : u[f];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int bx = c & 1, by = (c >> 1) & 1, bz = c >> 2;
      float d = 0.0f;
      if (ls.dtype == kU8) {
        unsigned w4[F / 4];
        load_codes<F>(r, base, off[c], w4);
#pragma unroll
        for (int q = 0; q < F / 4; ++q)
#pragma unroll
          for (int b = 0; b < 4; ++b) d = fmaf(us[4 * q + b], (float)((w4[q] >> (8 * b)) & 0xffu), d);
      } else if (ls.dtype == kF16) {
#pragma unroll
        for (int q = 0; q < F / 8; ++q) {
          const h8 hv = __builtin_bit_cast(h8, load16(r, base * 2u + 16u * q, off[c] * 2u));
#pragma unroll
          for (int j = 0; j < 8; ++j) d = fmaf(us[8 * q + j], (float)hv[j], d);
        }
      } else {
#pragma unroll
        for (int q = 0; q < F / 4; ++q) {
          const float4 v = __builtin_bit_cast(float4, load16(r, base * 4u + 16u * q, off[c] * 4u));
          d = fmaf(us[4 * q], v.x, fmaf(us[4 * q + 1], v.y, fmaf(us[4 * q + 2], v.z, fmaf(us[4 * q + 3], v.w, d))));
        }
      }
      d *= kw;
      g[0] = fmaf(DX[bx] * Y[by] * Z[bz], d, g[0]);
      g[1] = fmaf(X[bx] * DY[by] * Z[bz], d, g[1]);
      g[2] = fmaf(X[bx] * Y[by] * DZ[bz], d, g[2]);
    }
  }
}

// latent_vjp for an FP16 network on an FP16 grid: the row's FP16 latent
// entries u are dotted with each corner's FP16 vector two channels per
// v_dot2_f32_f16 (FP32 accumulation, the products exact as in latent_vjp),
// and the trilinear derivative is taken from the eight corner sums by
// differences along each axis: dy/dp_x = dx * sum over (y, z) of
// Y Z (d[1,y,z] - d[0,y,z]), likewise for y and z.
template <int F>
__device__ inline void latent_vjp_h(const LatentSrc& ls, float px, float py, float pz, const h2* u2, float g[3]) {
  int ix, iy, iz;
  float fx, fy, fz, dx, dy, dz;
  axis_cell(px, ls.R, ix, fx, dx);
  axis_cell(py, ls.R, iy, fy, dy);
  axis_cell(pz, ls.R, iz, fz, dz);
  const float X[2] = {1.0f - fx, fx}, Y[2] = {1.0f - fy, fy}, Z[2] = {1.0f - fz, fz};
  const float yz[4] = {Y[0] * Z[0], Y[1] * Z[0], Y[0] * Z[1], Y[1] * Z[1]};  // [by + 2 bz]
  const float xz[4] = {X[0] * Z[0], X[1] * Z[0], X[0] * Z[1], X[1] * Z[1]};  // [bx + 2 bz]
  const float xy[4] = {X[0] * Y[0], X[1] * Y[0], X[0] * Y[1], X[1] * Y[1]};  // [bx + 2 by]
  const unsigned R = (unsigned)ls.R;
  const unsigned sx = F, sy = R * F, sz = R * R * F;
  const unsigned base = (unsigned)iz * sz + (unsigned)iy * sy + (unsigned)ix * sx;
  unsigned off[8];
  corner_offsets(sx, sy, sz, off);
#pragma unroll
  for (int key = 0; key < 2; ++key) {
    const void* grid = key == 0 ? ls.g0 : ls.g1;
    if (key == 1 && !grid) break;
    const __amdgpu_buffer_rsrc_t r = grid_rsrc(grid, ls.bytes);
    float d[8];  // corner c = bx + 2 by + 4 bz
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < F / 8; ++q) {
        const h8 hv = __builtin_bit_cast(h8, load16(r, base * 2u + 16u * q, off[c] * 2u));
#pragma unroll
        for (int j = 0; j < 4; ++j) s = __builtin_amdgcn_fdot2(u2[4 * q + j], h2{hv[2 * j], hv[2 * j + 1]}, s, false);
      }
      d[c] = s;
    }
    float tx = 0.0f, ty = 0.0f, tz = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int lo = i & 1, hi = i >> 1;
      tx = fmaf(yz[i], d[1 + 2 * lo + 4 * hi] - d[2 * lo + 4 * hi], tx);
      ty = fmaf(xz[i], d[lo + 2 + 4 * hi] - d[lo + 4 * hi], ty);
      tz = fmaf(xy[i], d[lo + 2 * hi + 4] - d[lo + 2 * hi], tz);
    }
    const float kw = key == 0 ? ls.w0 : ls.w1;
    g[0] = fmaf(kw * dx, tx, g[0]);
    g[1] = fmaf(kw * dy, ty, g[1]);
    g[2] = fmaf(kw * dz, tz, g[2]);
  }
}

// The lane's gradient dy/dp from its row u = dy/d(input row) (left by
// mlp_tile_adj) and the Jacobian of the input row at p: x, y, z directly;
// Fourier columns d sin(w p_a)/dp_a = w cos(w p_a), d cos(w p_a)/dp_a =
// -w sin(w p_a) with w = pi 2^k (Sec. 3, Eq. 1-2); latent columns through
// latent_vjp.
template <class CF>
__device__ inline void input_vjp(const typename CF::E* row, const LatentSrc& ls, float px, float py, float pz,
                                 float g[3]) {
  using G = typename CF::G;
  constexpr int F = CF::F, L = CF::L;
  float u[G::KROW];
  if constexpr (CF::P == kF32) {
    const float4* src = reinterpret_cast<const float4*>(row);
#pragma unroll
    for (int q = 0; q < G::KROW / 4; ++q) {
      const float4 v = src[q];
      u[4 * q] = v.x;
      u[4 * q + 1] = v.y;
      u[4 * q + 2] = v.z;
      u[4 * q + 3] = v.w;
    }
  } else {
    using V8 = typename PrecT<CF::P>::VA;
    const V8* src = reinterpret_cast<const V8*>(row);
#pragma unroll
    for (int q = 0; q < G::KROW / 8; ++q) {
      const V8 v = src[q];
#pragma unroll
      for (int j = 0; j < 8; ++j) u[8 * q + j] = (float)v[j];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) g[a] = u[G::KMAIN + a];
  const float pp[3] = {px, py, pz};
  // sin and cos of each octave: exact phases on the FP32 path; octave 0 and
  // the double-angle recurrence (g = 2 cos) on the reduced-precision paths,
  // as the forward features are built there
  float sd[3], gd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sd[a] = sin_rev(0.5f * pp[a]);
    gd[a] = 2.0f * cos_rev(0.5f * pp[a]);
  }
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const float wk = kPi * (float)(1 << k);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float s, c;
      if constexpr (CF::P == kF32) {
        const float ph = pp[a] * (float)(1 << k) * 0.5f;
        s = sin_rev(ph);
        c = cos_rev(ph);
      } else {
        s = sd[a];
        c = 0.5f * gd[a];
        if (k + 1 < L) {
          sd[a] = sd[a] * gd[a];
          gd[a] = fmaf(gd[a], gd[a], -2.0f);
        }
      }
      g[a] = fmaf(wk, fmaf(u[F + 3 * k + a], c, -u[F + 3 * L + 3 * k + a] * s), g[a]);
    }
  }
  if constexpr (CF::P == kF16 && CF::GK == 1) {  // FP16 network on an FP16 grid
    latent_vjp_h<F>(ls, px, py, pz, reinterpret_cast<const h2*>(row), g);
  } else {
    latent_vjp<F>(ls, px, py, pz, u, g);
  }
}

}  // namespace fvsrn_detail
