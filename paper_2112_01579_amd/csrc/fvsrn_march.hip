// Per-precision instantiation and dispatch of the render and point kernels
// (compiled once per precision with FVSRN_PREC = 0 FP32, 1 FP16, 2 BF16);
// the adjoint shading mode lives in fvsrn_adjoint.hip.
#include "fvsrn_march.hpp"

#ifndef FVSRN_PREC
#error "FVSRN_PREC must be defined (0 FP32, 1 FP16, 2 BF16)"
#endif

namespace fvsrn_detail {

namespace {

template <int C, int F, int L, int ACT, int MODE, int GK>
struct Entry {
  using CF = Cfg<FVSRN_PREC, C, F, L, ACT, GK>;
  static int render(const NetDev& nd, const TFDev& tf, const ViewBatch& vb, const MarchDev& m, float* out,
                    unsigned long long* stats, hipStream_t st) {
    return launch_render_t<CF, MODE>(nd, tf, vb, m, out, stats, st);
  }
  static int points(const NetDev& nd, const float* xyz, long long n, int key, float key_w, float* out_d,
                    float* out_g, hipStream_t st) {
    // predicted gradients use the value-mode kernel (its out_g holds outputs 1..3)
    return launch_points_t<CF, MODE == kShadeFwd ? kShadeFwd : kShadeNone>(nd, xyz, n, key, key_w, out_d, out_g, st);
  }
};

// Gradient modes are compiled for every precision; central differences and
// predicted gradients for the sine activation only.

// The FP16 network has separate instantiations for FP32 (generic), FP16 and
// uint8 latent grids, the BF16 network for the generic path and FP16 grids.
#if FVSRN_PREC == 1
#define FV_G16S(X, C, F, L, ACT, MODE) X(C, F, L, ACT, MODE, 0) X(C, F, L, ACT, MODE, 1) X(C, F, L, ACT, MODE, 2)
#elif FVSRN_PREC == 2
#define FV_G16S(X, C, F, L, ACT, MODE) X(C, F, L, ACT, MODE, 0) X(C, F, L, ACT, MODE, 1)
#else
#define FV_G16S(X, C, F, L, ACT, MODE) X(C, F, L, ACT, MODE, 0)
#endif

#define FV_NETS(X, ACT, MODE)           \
  FV_G16S(X, 32, 8, 4, ACT, MODE)       \
  FV_G16S(X, 32, 16, 8, ACT, MODE)      \
  FV_G16S(X, 48, 8, 4, ACT, MODE)       \
  FV_G16S(X, 48, 16, 8, ACT, MODE)

#define FV_ALL(X)                    \
  FV_NETS(X, kSine, kShadeNone)      \
  FV_NETS(X, kSnakeAlt, kShadeNone)  \
  FV_NETS(X, kIdentity, kShadeNone)

#define FV_ALL_GRAD(X)              \
  FV_NETS(X, kSine, kShadeFwd)      \
  FV_NETS(X, kSnakeAlt, kShadeFwd)  \
  FV_NETS(X, kIdentity, kShadeFwd)

// Further shapes, sine activation, unshaded and forward mode: width 64, and
// latent channels and Fourier octaves chosen independently, (16, 4), (8, 8).
#define FV_NETS_EXT(X, MODE)                                                           \
  FV_G16S(X, 32, 16, 4, kSine, MODE) FV_G16S(X, 32, 8, 8, kSine, MODE)               \
  FV_G16S(X, 48, 16, 4, kSine, MODE) FV_G16S(X, 48, 8, 8, kSine, MODE)               \
  FV_G16S(X, 64, 8, 4, kSine, MODE) FV_G16S(X, 64, 16, 8, kSine, MODE)               \
  FV_G16S(X, 64, 16, 4, kSine, MODE) FV_G16S(X, 64, 8, 8, kSine, MODE)

#define FV_ALL_FD(X) FV_NETS(X, kSine, kShadeFD)
#define FV_ALL_PRED(X) FV_NETS(X, kSine, kShadePred)

}  // namespace

#define FV_PASTE2(a, b) a##b
#define FV_PASTE(a, b) FV_PASTE2(a, b)

int FV_PASTE(launch_render_p, FVSRN_PREC)(const NetDev& nd, const TFDev& tf, const ViewBatch& vb, const MarchDev& m,
                                          float* out, unsigned long long* stats, void* stream) {
  if (nd.fmat) return FV_PASTE(launch_render_rff_p, FVSRN_PREC)(nd, tf, vb, m, out, stats, stream);
  if (nd.time_enc != 0) return FV_PASTE(launch_render_time_p, FVSRN_PREC)(nd, tf, vb, m, out, stats, stream);
  if (m.phong && m.grad_mode == 3) return FV_PASTE(launch_render_adj_p, FVSRN_PREC)(nd, tf, vb, m, out, stats, stream);
  const int mode = !m.phong ? kShadeNone : (m.grad_mode == 1 ? kShadeFD : (m.grad_mode == 2 ? kShadePred : kShadeFwd));
  // packed FP16 gathers for an FP16 network on an FP16 or uint8 grid
  const int gk = FVSRN_PREC == 0 ? 0
                 : FVSRN_PREC == 2 ? (nd.grid_f16 && !nd.grid_u8 ? 1 : 0)
                                   : (nd.grid_u8 ? 2 : (nd.grid_f16 ? 1 : 0));
  const hipStream_t st = (hipStream_t)stream;
#define X(C_, F_, L_, ACT_, MODE_, GK_)                                                           \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_ && nd.act == ACT_ && mode == MODE_ && gk == GK_) \
    return Entry<C_, F_, L_, ACT_, MODE_, GK_>::render(nd, tf, vb, m, out, stats, st);
  FV_ALL(X)
  FV_ALL_PRED(X)
  FV_NETS_EXT(X, kShadeNone)
  FV_ALL_GRAD(X)
  FV_ALL_FD(X)
  FV_NETS_EXT(X, kShadeFwd)
#undef X
  return 1;
}

int FV_PASTE(launch_points_p, FVSRN_PREC)(const NetDev& nd, const float* xyz, long long n, int key, float key_w,
                                          float* out_d, float* out_g, int gmode, void* stream) {
  if (nd.fmat) return FV_PASTE(launch_points_rff_p, FVSRN_PREC)(nd, xyz, n, key, key_w, out_d, out_g, gmode, stream);
  if (nd.time_enc != 0)
    return FV_PASTE(launch_points_time_p, FVSRN_PREC)(nd, xyz, n, key, key_w, out_d, out_g, gmode, stream);
  if (out_g && gmode == 3) return FV_PASTE(launch_points_adj_p, FVSRN_PREC)(nd, xyz, n, key, key_w, out_d, out_g, stream);
  // gmode 2: a 4-output network's own gradient, from the value-mode kernel
  const int mode = (out_g != nullptr && gmode == 0) ? kShadeFwd : kShadeNone;
  // packed FP16 gathers for an FP16 network on an FP16 or uint8 grid
  const int gk = FVSRN_PREC == 0 ? 0
                 : FVSRN_PREC == 2 ? (nd.grid_f16 && !nd.grid_u8 ? 1 : 0)
                                   : (nd.grid_u8 ? 2 : (nd.grid_f16 ? 1 : 0));
  const hipStream_t st = (hipStream_t)stream;
#define X(C_, F_, L_, ACT_, MODE_, GK_)                                                           \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_ && nd.act == ACT_ && mode == MODE_ && gk == GK_) \
    return Entry<C_, F_, L_, ACT_, MODE_, GK_>::points(nd, xyz, n, key, key_w, out_d, out_g, st);
  FV_ALL(X)
  FV_NETS_EXT(X, kShadeNone)
  FV_ALL_GRAD(X)
  FV_NETS_EXT(X, kShadeFwd)
#undef X
  return 1;
}

}  // namespace fvsrn_detail
