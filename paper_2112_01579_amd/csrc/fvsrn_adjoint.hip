// Adjoint (reverse-mode) gradient shading and point gradients (Sec. 6),
// compiled once per precision with FVSRN_PREC = 0 FP32, 1 FP16 or 2 BF16. The layer
// count is a template parameter (the saved activation derivatives are
// registers), instantiated for H = 1..8 and the sine activation; above four
// layers the first ones are evaluated twice (see mlp_tile_adj).
#include "fvsrn_march.hpp"

#ifndef FVSRN_PREC
#error "FVSRN_PREC must be defined (0 FP32, 1 FP16, 2 BF16)"
#endif

namespace fvsrn_detail {

namespace {

constexpr int kAdjMaxLayers = 8;

template <int C, int F, int L, int GK, int HH>
struct AdjEntry {
  using CF = Cfg<FVSRN_PREC, C, F, L, kSine, GK>;
  static int render(const NetDev& nd, const TFDev& tf, const ViewBatch& vb, const MarchDev& m, float* out,
                    unsigned long long* stats, hipStream_t st) {
    return launch_render_t<CF, kShadeAdj, HH>(nd, tf, vb, m, out, stats, st);
  }
  static int points(const NetDev& nd, const float* xyz, long long n, int key, float key_w, float* out_d,
                    float* out_g, hipStream_t st) {
    return launch_points_t<CF, kShadeAdj, HH>(nd, xyz, n, key, key_w, out_d, out_g, st);
  }
};

#define FV_ADJ_H(X, C, F, L, GK)                                                             \
  X(C, F, L, GK, 1) X(C, F, L, GK, 2) X(C, F, L, GK, 3) X(C, F, L, GK, 4) X(C, F, L, GK, 5) \
  X(C, F, L, GK, 6) X(C, F, L, GK, 7) X(C, F, L, GK, 8)
#if FVSRN_PREC == 1
#define FV_ADJ_G(X, C, F, L) FV_ADJ_H(X, C, F, L, 0) FV_ADJ_H(X, C, F, L, 1) FV_ADJ_H(X, C, F, L, 2)
#else
#define FV_ADJ_G(X, C, F, L) FV_ADJ_H(X, C, F, L, 0)
#endif
#define FV_ADJ_ALL(X)         \
  FV_ADJ_G(X, 32, 8, 4)       \
  FV_ADJ_G(X, 32, 16, 8)      \
  FV_ADJ_G(X, 48, 8, 4)       \
  FV_ADJ_G(X, 48, 16, 8)

}  // namespace

#define FV_PASTE2(a, b) a##b
#define FV_PASTE(a, b) FV_PASTE2(a, b)

int FV_PASTE(launch_render_adj_p, FVSRN_PREC)(const NetDev& nd, const TFDev& tf, const ViewBatch& vb,
                                              const MarchDev& m, float* out, unsigned long long* stats,
                                              void* stream) {
  if (nd.act != kSine || nd.H > kAdjMaxLayers) return 1;
  const int gk = FVSRN_PREC != 1 ? 0 : (nd.grid_u8 ? 2 : (nd.grid_f16 ? 1 : 0));
  const hipStream_t st = (hipStream_t)stream;
#define X(C_, F_, L_, GK_, H_)                                                        \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_ && gk == GK_ && nd.H == H_) \
    return AdjEntry<C_, F_, L_, GK_, H_>::render(nd, tf, vb, m, out, stats, st);
  FV_ADJ_ALL(X)
#undef X
  return 1;
}

int FV_PASTE(launch_points_adj_p, FVSRN_PREC)(const NetDev& nd, const float* xyz, long long n, int key,
                                              float key_w, float* out_d, float* out_g, void* stream) {
  if (nd.act != kSine || nd.H > kAdjMaxLayers) return 1;
  const int gk = FVSRN_PREC != 1 ? 0 : (nd.grid_u8 ? 2 : (nd.grid_f16 ? 1 : 0));
  const hipStream_t st = (hipStream_t)stream;
#define X(C_, F_, L_, GK_, H_)                                                        \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_ && gk == GK_ && nd.H == H_) \
    return AdjEntry<C_, F_, L_, GK_, H_>::points(nd, xyz, n, key, key_w, out_d, out_g, st);
  FV_ADJ_ALL(X)
#undef X
  return 1;
}

}  // namespace fvsrn_detail
