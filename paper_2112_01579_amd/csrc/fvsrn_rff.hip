// Networks whose Fourier features come from a general matrix (Sec. 3:
// random Fourier features, rows drawn from N(0, (2 pi sigma)^2)), compiled
// once per precision with FVSRN_PREC = 0 FP32, 1 FP16 or 2 BF16, sine
// activation: the unshaded render and point densities, forward-mode density
// gradients and Phong shading from them, Phong shading from central
// differences and, for four-output networks, from the predicted gradient.
#include "fvsrn_march.hpp"

#ifndef FVSRN_PREC
#error "FVSRN_PREC must be defined (0 FP32, 1 FP16, 2 BF16)"
#endif

namespace fvsrn_detail {

namespace {

template <int C, int F, int L, int GK>
struct RffEntry {
  using CF = Cfg<FVSRN_PREC, C, F, L, kSine, GK, 0, 1>;
  static int render(const NetDev& nd, const TFDev& tf, const ViewBatch& vb, const MarchDev& m, float* out,
                    unsigned long long* stats, hipStream_t st) {
    if (!m.phong) return launch_render_t<CF, kShadeNone>(nd, tf, vb, m, out, stats, st);
    if (m.grad_mode == 0) return launch_render_t<CF, kShadeFwd>(nd, tf, vb, m, out, stats, st);
    if (m.grad_mode == 1) return launch_render_t<CF, kShadeFD>(nd, tf, vb, m, out, stats, st);
    if (m.grad_mode == 2) return launch_render_t<CF, kShadePred>(nd, tf, vb, m, out, stats, st);
    return 1;
  }
  static int points(const NetDev& nd, const float* xyz, long long n, int key, float key_w, float* out_d,
                    float* out_g, int gmode, hipStream_t st) {
    if (!out_g) return launch_points_t<CF, kShadeNone>(nd, xyz, n, key, key_w, out_d, nullptr, st);
    if (gmode == 0) return launch_points_t<CF, kShadeFwd>(nd, xyz, n, key, key_w, out_d, out_g, st);
    // a four-output network's own gradient (outputs 1..3) from the value-mode kernel
    if (gmode == 2) return launch_points_t<CF, kShadeNone>(nd, xyz, n, key, key_w, out_d, out_g, st);
    return 1;
  }
};

#if FVSRN_PREC == 1
#define FV_RFF_G(X, C, F, L) X(C, F, L, 0) X(C, F, L, 1) X(C, F, L, 2)
#else
#define FV_RFF_G(X, C, F, L) X(C, F, L, 0)
#endif
#define FV_RFF_ALL(X)        \
  FV_RFF_G(X, 32, 8, 4)      \
  FV_RFF_G(X, 32, 16, 8)     \
  FV_RFF_G(X, 48, 8, 4)      \
  FV_RFF_G(X, 48, 16, 8)

}  // namespace

#define FV_PASTE2(a, b) a##b
#define FV_PASTE(a, b) FV_PASTE2(a, b)

int FV_PASTE(launch_render_rff_p, FVSRN_PREC)(const NetDev& nd, const TFDev& tf, const ViewBatch& vb,
                                              const MarchDev& m, float* out, unsigned long long* stats,
                                              void* stream) {
  if (nd.act != kSine || nd.time_enc != 0) return 1;
  const int gk = FVSRN_PREC != 1 ? 0 : (nd.grid_u8 ? 2 : (nd.grid_f16 ? 1 : 0));
  const hipStream_t st = (hipStream_t)stream;
#define X(C_, F_, L_, GK_)                                    \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_ && gk == GK_) \
    return RffEntry<C_, F_, L_, GK_>::render(nd, tf, vb, m, out, stats, st);
  FV_RFF_ALL(X)
#undef X
  return 1;
}

int FV_PASTE(launch_points_rff_p, FVSRN_PREC)(const NetDev& nd, const float* xyz, long long n, int key,
                                              float key_w, float* out_d, float* out_g, int gmode, void* stream) {
  if (nd.act != kSine || nd.time_enc != 0) return 1;
  const int gk = FVSRN_PREC != 1 ? 0 : (nd.grid_u8 ? 2 : (nd.grid_f16 ? 1 : 0));
  const hipStream_t st = (hipStream_t)stream;
#define X(C_, F_, L_, GK_)                                    \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_ && gk == GK_) \
    return RffEntry<C_, F_, L_, GK_>::points(nd, xyz, n, key, key_w, out_d, out_g, gmode, st);
  FV_RFF_ALL(X)
#undef X
  return 1;
}

}  // namespace fvsrn_detail
