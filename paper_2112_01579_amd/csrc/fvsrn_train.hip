// Training step of the fV-SRN (world-space fitting with L1 loss and Adam,
// Sec. 3 and Sec. 5): FP32 parameters, gradients and Adam; the network's
// forward and backward passes in FP32 (fwd_bwd_kernel) or FP16
// (fwd_bwd_h_kernel, further below) MFMA.
//
// fwd_bwd_kernel: each wave takes chunks of S = 16 points (fixed,
// grid-independent assignment: chunk c goes to wave c mod n_waves; one MFMA
// N-tile per chunk keeps the per-wave LDS small enough for six waves per CU).
// Per chunk:
//   1. the wave's 64 lanes write the chunk's 16 input rows to LDS, four lanes
//      per point (write_row_quad);
//   2. forward through the layers on 16x16x4 FP32 MFMA, keeping every
//      pre-activation a_i in LDS (sample-major);
//   3. output sigmoid, loss and dL/dy (for a 4-output network fitted with
//      gradient targets, also the L1 terms of the predicted gradient, Sec. 6);
//   4. backward: delta_i = (W_{i+1}^T delta_{i+1}) * act'(a_i) on MFMA with
//      transposed weight fragments; dW_i = delta_i h_i^T as an MFMA GEMM over
//      the chunk's samples (A = delta, B = layer input, both read from LDS);
//   5. dL/dz = W_0[:, latent]^T delta_0, stored per point with the point's
//      latent cell (and the cell's point count).
// dW tiles are summed per wave over its chunks (no atomics, so dW is bitwise
// reproducible): the tiles that fit stay in registers, the hidden layers'
// bias gradients in a small LDS area, the rest are added into the wave's
// workspace slice; each wave writes its sums to its slice at the end.
// slice_sum_kernel and gather_kernel then sum the slices in a fixed order
// into the packed gradient; adam_kernel applies the update.
// The latent gradient is gathered, not scattered: the points are
// counting-sorted by cell (the cell scan kernels, bin_points_kernel) and every
// grid vertex sums the trilinear-weighted dL/dz of the points in its (up to)
// eight cells, in two passes (cell_partials_kernel, vertex_sum_kernel) or one
// (latent_grad_kernel), with plain stores.
#include <cmath>
#include <mutex>

#include "fvsrn_net.hpp"

namespace fvsrn_detail {

namespace {

// Fixed number of waves (a deterministic partition, so a fixed dW summation
// order). At c = 48 a wave's slice holds no register-resident tiles and is
// read and written back for every chunk; 1024 slices of the 4 x 48 network
// (about 5.6 MB per XCD) stay closer to the L2 than 2048 (0.380 -> 0.354 ms
// per 2^18-point FP16 step, 0.464 -> 0.443 FP32; 512 waves lose occupancy).
constexpr int kTrainMaxWaves = 2048;
constexpr int kTrainMaxWaves48 = 1024;
constexpr int kTrainWavesPerBlock = 8;

template <int C, int F, int L, int ACT, int TE = 0, int FM = 0>
struct TrainCfg {
  using CF = Cfg<kF32, C, F, L, ACT, 0, TE, FM>;
  using G = typename CF::G;
  static constexpr int S = 16;                      // points per wave chunk (one N-tile)
  static constexpr int NTC = S / 16;
  static constexpr int MT = G::MT;
  static constexpr int NK0 = (G::KROW + 15) / 16;   // N-tiles of layer 0's input row
  static constexpr int AS = C + 4;                  // sample-major row stride (floats)
  static constexpr int ZS = 20;                     // latent-gradient row stride
  // per-wave LDS (bytes)
  static constexpr int FEAT = S * G::ROW * 4;
  __host__ __device__ static int abuf_bytes(int H) { return H * S * AS * 4; }
  static constexpr int DBUF = S * AS * 4;
  static constexpr int DY = 64 * 4;                 // dL/dy [output][sample]
  static_assert(4 * S <= 64, "four outputs of S samples must fit the dL/dy buffer");
  static constexpr int ZBUF = S * ZS * 4;
  static constexpr int BACC = MT * 4 * 16;          // one layer's bias sums: [M-tile][row group] f4
  __host__ __device__ static int wave_bytes(int H) { return FEAT + abuf_bytes(H) + DBUF + DY + ZBUF + (H - 1) * BACC; }
  // The backward pass needs W^T. For c = 32 a transposed copy of each hidden
  // layer and of W_0's latent columns is staged once per workgroup (14 KiB at
  // H = 4: one wave of seven fewer per CU, but lane-contiguous reads); wider
  // networks read W^T from the forward fragments instead (strided reads with
  // bank conflicts, but for c = 48 the copy would cost a quarter of the
  // waves: measured 0.80 -> 0.62 ms per 2^18-point Adam step, while c = 32
  // measured 0.415 with the copy against 0.433 without).
  static constexpr bool kBackCopy = C == 32;
  static constexpr int WB = MT * 4 * MT * 64 * 4;   // one hidden layer's W^T
  static constexpr int WZ = 4 * MT * 64 * 4;        // latent columns of W_0, transposed
  __host__ __device__ static int back_bytes(int H) { return kBackCopy ? (H - 1) * WB + WZ : 0; }
  __host__ __device__ static int block_bytes(int H, int waves) {
    return G::weight_bytes(H) + back_bytes(H) + waves * wave_bytes(H);
  }
  // workspace slice (floats)
  __host__ __device__ static int tiles(int H) { return MT * NK0 + (H - 1) * MT * MT + MT + (H - 1) * MT; }
  // after the tiles: per-lane partials of the four output biases, then of the loss
  __host__ __device__ static int slice(int H) { return tiles(H) * 256 + 5 * 64; }
  __host__ __device__ static int tile_l0(int mo, int nk) { return mo * NK0 + nk; }
  __host__ __device__ static int tile_h(int H, int i, int mo, int nk) { return MT * NK0 + (i - 1) * MT * MT + mo * MT + nk; }
  __host__ __device__ static int tile_out(int H, int nk) { return MT * NK0 + (H - 1) * MT * MT + nk; }
  __host__ __device__ static int tile_bias(int H, int i, int mt) { return MT * NK0 + (H - 1) * MT * MT + MT + (i - 1) * MT + mt; }
};

// Sum over the 16 lanes of this lane's row (lanes with the same lane >> 4),
// in DPP steps that every lane takes alike: pairs (quad_perm 1 0 3 2), quads
// (quad_perm 2 3 0 1), halves of the row (row_half_mirror), the row
// (row_mirror); every lane of the row receives the same sum.
__device__ inline float dpp_add(float v, int ctrl_sel) {
  int t;
  switch (ctrl_sel) {
    case 0: t = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false); break;
    case 1: t = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false); break;
    case 2: t = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false); break;
    default: t = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false); break;
  }
  return v + __builtin_bit_cast(float, t);
}

__device__ inline f4 row16_sum(f4 v) {
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = dpp_add(v[j], st);
  return v;
}

template <int ACT>
__device__ inline float act_d(float a) {  // d act / d x at pre-activation a (revolutions for periodic acts)
  if constexpr (ACT == kSine) return cos_rev(a);
  else if constexpr (ACT == kSnakeAlt) return 0.5f + sin_rev(2.0f * a);
  else return 1.0f;
}

// Backward weight fragments: W_i^T for i = 1..H-1 and the latent columns of W_0
// transposed. The forward fragments hold W scaled by 1/(2 pi) for periodic
// activations; the transposed ones here are unscaled, since the chain rule in
// x units is delta_h = W^T (delta_a).
template <class TC, int ACT>
__device__ void stage_backward(const NetDev& nd, char* p) {
  constexpr int C = TC::CF::C, F = TC::CF::F, L = TC::CF::L, MT = TC::MT;
  const int H = nd.H, K0 = TC::G::K0IN;
  const float* w = nd.weights;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = 1; i < H; ++i) {
    const float* Wi = w + (long long)C * K0 + C + (long long)(i - 1) * (C * C + C);
    float* WB = reinterpret_cast<float*>(p + (i - 1) * TC::WB);
    for (int e = tid; e < MT * 4 * MT * 64; e += nt) {
      const int lane = e & 63, q = (e >> 6) % (4 * MT), mk = (e >> 6) / (4 * MT);
      const int o = 16 * (q / 4) + 4 * (lane >> 4) + (q % 4);
      WB[e] = Wi[o * C + 16 * mk + (lane & 15)];
    }
  }
  float* WZ = reinterpret_cast<float*>(p + (H - 1) * TC::WB);
  for (int e = tid; e < 4 * MT * 64; e += nt) {
    const int lane = e & 63, q = e >> 6, m = lane & 15;
    const int o = 16 * (q / 4) + 4 * (lane >> 4) + (q % 4);
    WZ[e] = m < F ? w[(long long)o * K0 + 3 + m] : 0.0f;
  }
}

// Keyframe pair of time t (Sec. 8): the time clamped to the key range,
// linear between the neighbouring keyframes; key = 0, kw = 0 for one keyframe.
__device__ inline void key_pair(const KeyTimes& kt, int K, float t, int& key, float& kw) {
  key = 0;
  kw = 0.0f;
  if (K > 1) {
    if (t <= kt.t[0]) {
      key = 0;
      kw = 0.0f;
    } else if (t >= kt.t[K - 1]) {
      key = K - 2;
      kw = 1.0f;
    } else {
      while (key + 1 < K - 1 && kt.t[key + 1] <= t) ++key;
      kw = (t - kt.t[key]) / (kt.t[key + 1] - kt.t[key]);
    }
  }
}

// The input rows of a chunk's 16 points (Sec. 3: latent, Fourier features,
// x y z 1), built by all 64 lanes: lane q of quad p writes channels
// [q F/4, (q + 1) F/4) of point p's latent vector (its corner loads are one
// quarter of the point's), octaves q, q + 4, ... of its Fourier features, and
// lane 0 of the quad the tail and the zero padding. Octave phases are exact
// powers of two times p (no double-angle recurrence); FP16/BF16 rows hold
// 2 cos like the render's. The latent sums run over the corners in the
// per-lane gather's order, so FP32 rows are the same bits. FP32 latent grids
// (the training parameters).
template <class CF>
__device__ inline void write_row_quad(typename CF::E* row, const LatentSrc& ls, int q, float px, float py, float pz) {
  using G = typename CF::G;
  using E = typename CF::E;
  constexpr int F = CF::F, L = CF::L, FQ = F / 4;
  int ix, iy, iz;
  float fx, fy, fz;
  axis_cell(px, ls.R, ix, fx);
  axis_cell(py, ls.R, iy, fy);
  axis_cell(pz, ls.R, iz, fz);
  const float x0 = 1.0f - fx, x1 = fx, y0 = 1.0f - fy, y1 = fy, z0 = 1.0f - fz, z1 = fz;
  const unsigned R = (unsigned)ls.R;
  const unsigned sx = F, sy = R * F, sz = R * R * F;
  const unsigned base = (unsigned)iz * sz + (unsigned)iy * sy + (unsigned)ix * sx;
  unsigned off[8];
  corner_offsets(sx, sy, sz, off);
  const float w[8] = {x0 * y0 * z0, x1 * y0 * z0, x0 * y1 * z0, x1 * y1 * z0,
                      x0 * y0 * z1, x1 * y0 * z1, x0 * y1 * z1, x1 * y1 * z1};
  float z[FQ];
#pragma unroll
  for (int j = 0; j < FQ; ++j) z[j] = 0.0f;
#pragma unroll
  for (int key = 0; key < 2; ++key) {
    const void* g = key == 0 ? ls.g0 : ls.g1;
    if (key == 1 && !g) break;
    const float kw = key == 0 ? ls.w0 : ls.w1;
    const __amdgpu_buffer_rsrc_t r = grid_rsrc(g, ls.bytes);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float wc = w[c] * kw;
      if constexpr (FQ == 4) {
        const float4 v = __builtin_bit_cast(float4, load16(r, base * 4u + 16u * (unsigned)q, off[c] * 4u));
        z[0] = fmaf(wc, v.x, z[0]);
        z[1] = fmaf(wc, v.y, z[1]);
        z[2] = fmaf(wc, v.z, z[2]);
        z[3] = fmaf(wc, v.w, z[3]);
      } else {
        static_assert(FQ == 2, "F = 8 or 16");
        const float2 v = __builtin_bit_cast(float2, load8(r, base * 4u + 8u * (unsigned)q, off[c] * 4u));
        z[0] = fmaf(wc, v.x, z[0]);
        z[1] = fmaf(wc, v.y, z[1]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < FQ; ++j) row[FQ * q + j] = to_e<E>(z[j]);
  constexpr float cs = CF::P == kF32 ? 1.0f : 2.0f;  // scale of the cosine block
  const float pp[3] = {px, py, pz};
#pragma unroll
  for (int i = 0; i < L / 4; ++i) {
    const int k = q + 4 * i;
    const float sc = (float)(1 << k) * 0.5f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float ph = pp[a] * sc;
      row[F + 3 * k + a] = to_e<E>(sin_rev(ph));
      row[F + 3 * L + 3 * k + a] = to_e<E>(cs * cos_rev(ph));
    }
  }
  if (q == 0) {
#pragma unroll
    for (int j = G::KF; j < G::KMAIN; ++j) row[j] = to_e<E>(0.0f);
    row[G::KMAIN + 0] = to_e<E>(px);
    row[G::KMAIN + 1] = to_e<E>(py);
    row[G::KMAIN + 2] = to_e<E>(pz);
    row[G::KMAIN + 3] = to_e<E>(1.0f);
#pragma unroll
    for (int j = G::KMAIN + 4; j < G::KROW; ++j) row[j] = to_e<E>(0.0f);
  }
}

template <int C, int F, int L, int ACT, int TE, int FM>
__global__ __launch_bounds__(kTrainWavesPerBlock * 64) void fwd_bwd_kernel(NetDev nd, KeyTimes kt, const float* xyz,
                                                                            const float* times, long long n,
                                                                            const float* target,
                                                                            const float* target_grad, float gw3,
                                                      const float* dloss, float* dz_out, int* cell_out,
                                                      int* cell_count, int* rank_out, float* ws, int n_waves,
                                                      float inv_n) {
  using TC = TrainCfg<C, F, L, ACT, TE, FM>;
  using CF = typename TC::CF;
  using G = typename TC::G;
  using PR = PrecT<kF32>;
  constexpr int MT = TC::MT, AS = TC::AS, S = TC::S, NTC = TC::NTC;
  const int H = nd.H, NO = nd.NO;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  stage_weights<CF>(nd, smem);
  char* back = smem + G::weight_bytes(H);
  if constexpr (TC::kBackCopy) stage_backward<TC, ACT>(nd, back);
  __syncthreads();
  const int wave_l = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + wave_l;
  if (wave >= n_waves) return;
  const int g = lane >> 4, nn = lane & 15;
  char* wbase = back + TC::back_bytes(H) + wave_l * TC::wave_bytes(H);
  float* feat = reinterpret_cast<float*>(wbase);
  float* abuf = reinterpret_cast<float*>(wbase + TC::FEAT);
  float* dbuf = reinterpret_cast<float*>(wbase + TC::FEAT + TC::abuf_bytes(H));
  float* dy = reinterpret_cast<float*>(wbase + TC::FEAT + TC::abuf_bytes(H) + TC::DBUF);
  float* zbuf = reinterpret_cast<float*>(wbase + TC::FEAT + TC::abuf_bytes(H) + TC::DBUF + TC::DY);
  // bias gradients of the hidden layers, summed over the chunk's points in the
  // wave and accumulated here over its chunks ([layer][M-tile][row group])
  f4* bacc = reinterpret_cast<f4*>(wbase + TC::FEAT + TC::abuf_bytes(H) + TC::DBUF + TC::DY + TC::ZBUF);
  for (int e = lane; e < (H - 1) * MT * 4; e += kWave) bacc[e] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  float* slice = ws + (size_t)wave * TC::slice(H);
  const float* W0 = reinterpret_cast<const float*>(smem);
  const char* wout_p = smem + G::W0A + (H - 1) * G::HID;
  const float* WO = reinterpret_cast<const float*>(wout_p);
  const f4 b_out = *reinterpret_cast<const f4*>(wout_p + G::WOA);
  // output weights W_out[o][k] (unscaled) straight from global memory
  const float* w_out = nd.weights + (long long)C * G::K0IN + C + (long long)(H - 1) * (C * C + C);
  float loss_acc = 0.0f;
  f4 dbo_acc = {0.0f, 0.0f, 0.0f, 0.0f};
  // Without the copy, W^T from the forward A fragments. Hidden layer i holds W_i[o][k] * sc at
  // ((o / 16) 4MT + 4 (k / 16) + k % 4) 64 + 16 ((k % 16) / 4) + o % 16; the
  // backward A operand of lane (g, n) at step q, M-tile mk is W_i[o][k] with
  // o = 16 (q / 4) + 4 g + q % 4 and k = 16 mk + n. Layer 0's latent column m
  // sits at input-row column m. sc is the 1 / (2 pi) the forward fragments
  // carry for periodic activations; the deltas are multiplied by its inverse.
  const int wt_lane = (nn & 3) * kWave + 16 * (nn >> 2) + 4 * g;
  const int wz_lane = ((nn % G::Q0) * kWave + 16 * (nn / G::Q0) + 4 * g);
  const float inv_sc = ACT == kIdentity ? 1.0f : k2Pi;
  const long long nchunks = (n + S - 1) / S;
  bool first = true;
  // Branch-free on purpose: the stored value is always produced by a VALU
  // select, never by the MFMA directly. (A global store of an MFMA result
  // reached through a branch was issued without the wait states the result
  // needs and stored a partly written tile.) The first chunk's load reads
  // stale workspace and is discarded by the select.
  // A layer's running tile sums are loaded together before its gradient
  // MFMAs, so the loads are in flight meanwhile.
  auto load_tiles = [&](int t0, int cnt, f4* old) {
    for (int k = 0; k < cnt; ++k) old[k] = reinterpret_cast<const f4*>(slice + (t0 + k) * 256)[lane];
  };
  auto put_tile = [&](int tile, f4 old, f4 v) {
    f4 r;
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = first ? v[j] : old[j] + v[j];
    reinterpret_cast<f4*>(slice + tile * 256)[lane] = r;
  };
  // A chunk's positions, times and targets (or loss gradients) are loaded
  // one chunk ahead, after the input rows of the chunk before are built, so
  // that these HBM reads overlap its passes instead of preceding the gather.
  float npx, npy, npz, npt, ntg;
  auto load_point = [&](long long cc) {
    const long long j = cc * S + lane;
    npx = npy = npz = npt = ntg = 0.0f;
    if (lane < S && cc < nchunks && j < n) {
      npx = xyz[3 * j];
      npy = xyz[3 * j + 1];
      npz = xyz[3 * j + 2];
      if (times) npt = times[j];
      ntg = target ? target[j] : dloss[j];
    }
  };
  // For c = 32 the layer-0 weight-gradient tiles (the largest group) stay in
  // registers over the wave's chunks and go to the slice once at the end:
  // the same sums in the same order as the slice's read-modify-write.
  // So do the last hidden layer's, and at every width the output layer's.
  constexpr bool kResident0 = C == 32;
  constexpr int R0 = kResident0 ? MT : 1;  // layer-0 M-tiles held (the first one at c = 48)
  constexpr int NR0 = R0 * TC::NK0, NRO = MT, NRH = kResident0 ? MT * MT : 1;
  f4 acc0[NR0], accO[NRO], accH[NRH];
#pragma unroll
  for (int k = 0; k < NR0; ++k) acc0[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < NRO; ++k) accO[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < NRH; ++k) accH[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  load_point(wave);
  for (long long c = wave; c < nchunks; c += n_waves) {
    // lane l < S owns point c * S + l
    const long long idx = c * S + lane;
    const bool ok = lane < S && idx < n;
    const float px = npx, py = npy, pz = npz, pt = npt, tg = ntg;
    if constexpr (TE == 0 && FM == 0) {
      // quad lane >> 2 builds that point's row
      const int src = lane >> 2;
      const float qx = __shfl(px, src, 64), qy = __shfl(py, src, 64), qz = __shfl(pz, src, 64);
      if (nd.K == 1) {
        write_row_quad<CF>(feat + src * G::ROW, make_latent_src(nd, 0, 0.0f), lane & 3, qx, qy, qz);
      } else {
        // this point's keyframe pair (Sec. 8)
        int key;
        float kw;
        key_pair(kt, nd.K, __shfl(pt, src, 64), key, kw);
        write_row_quad<CF>(feat + src * G::ROW, make_latent_src(nd, key, kw), lane & 3, qx, qy, qz);
      }
    } else {
      // this point's keyframe pair (Sec. 8)
      int key;
      float kw;
      key_pair(kt, nd.K, pt, key, kw);
      float tfe[G::TIN > 0 ? G::TIN : 1];  // the point's time inputs (Sec. 8)
      if constexpr (G::TIN > 0) time_features<TE>(time_tau(pt, nd.t_lo, nd.t_hi, nd.t_scale), tfe);
      if (lane < S) {
        if (nd.K == 1) {
          write_features<CF, false>(feat + lane * G::ROW, make_latent_src(nd, 0, 0.0f), value_role(), px, py, pz,
                                    tfe, nd.fm);
        } else {
          // per-lane keyframes: the buffer loads of the gather then run once
          // per distinct keyframe present in the wave
          write_features<CF, false>(feat + lane * G::ROW, make_latent_src(nd, key, kw), value_role(), px, py, pz,
                                    tfe, nd.fm);
        }
      }
    }
    wave_lds_sync();
    load_point(c + n_waves);
    // ---------------- forward: store pre-activations a_i[s][o]
    f4 out = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int t = 0; t < NTC; ++t) {
      f4 acc[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < G::Q0; ++q) {
        const float b = feat[(16 * t + nn) * G::ROW + g * G::Q0 + q];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = PR::mma(W0[(mt * G::Q0 + q) * kWave + lane], b, acc[mt]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) *reinterpret_cast<f4*>(abuf + (16 * t + nn) * AS + 16 * mt + 4 * g) = acc[mt];
      const char* p = smem + G::W0A;
      for (int i = 1; i < H; ++i) {
        const float* WH = reinterpret_cast<const float*>(p);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA);
        f4 nacc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) nacc[mt] = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g);
#pragma unroll
        for (int q = 0; q < 4 * MT; ++q) {
          const float b = act_el<ACT, false>(acc[q / 4][q % 4], value_role());
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) nacc[mt] = PR::mma(WH[(mt * 4 * MT + q) * kWave + lane], b, nacc[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          acc[mt] = nacc[mt];
          *reinterpret_cast<f4*>(abuf + i * S * AS + (16 * t + nn) * AS + 16 * mt + 4 * g) = acc[mt];
        }
        p += G::HID;
      }
#pragma unroll
      for (int q = 0; q < 4 * MT; ++q) {
        const float b = act_el<ACT, false>(acc[q / 4][q % 4], value_role());
        out = PR::mma(WO[(t * 4 * MT + q) * kWave + lane], b, out);
      }
    }
    // ---------------- loss and dL/dy for this lane's own sample (lanes < S
    // hold its outputs in out[0..NO))
    const f4 yv = out + b_out;
    const float d = sigmoid_f(yv[0]);
    float gy = 0.0f;
    f4 dyo = {0.0f, 0.0f, 0.0f, 0.0f};
    if (ok) {
      if (target) {
        const float r = d - tg;
        loss_acc += fabsf(r);
        gy = (r > 0.0f ? 1.0f : (r < 0.0f ? -1.0f : 0.0f)) * inv_n;
        if (target_grad) {
          // predicted gradient (outputs 1..3) against its targets, weighted L1
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float rg = yv[1 + a] - target_grad[3 * idx + a];
            loss_acc += gw3 * fabsf(rg);
            dyo[1 + a] = (rg > 0.0f ? gw3 : (rg < 0.0f ? -gw3 : 0.0f)) * inv_n;
          }
        }
      } else {
        loss_acc += tg * d;
        gy = tg;
      }
    }
    dyo[0] = gy * d * (1.0f - d);
    dbo_acc += dyo;
    if (lane < S) {
#pragma unroll
      for (int o = 0; o < 4; ++o) dy[o * S + lane] = dyo[o];
    }
    wave_lds_sync();
    // ---------------- output layer weights: dW_H[o][k] = sum_s dy[o][s] h[k][s]
    const float* alast = abuf + (H - 1) * S * AS;

#pragma unroll
    for (int nk = 0; nk < MT; ++nk) {
      f4 dw = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < S / 4; ++q) {
        const int s = 4 * q + g;
        const float a = nn < NO ? dy[nn * S + s] : 0.0f;
        const float b = act_el<ACT, false>(alast[s * AS + 16 * nk + nn], value_role());
        dw = PR::mma(a, b, dw);
      }
      accO[nk] += dw;
    }
    // ---------------- backward through the activated layers
    f4 dh[NTC][MT];  // d L / d h_i in D layout, per N-tile
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) dh[t][mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      for (int o = 0; o < NO; ++o) {
        const float dys = dy[o * S + 16 * t + nn];
        const float* wr = w_out + o * C;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const f4 wo = {wr[16 * mt + 4 * g + 0], wr[16 * mt + 4 * g + 1], wr[16 * mt + 4 * g + 2],
                         wr[16 * mt + 4 * g + 3]};
          dh[t][mt] += wo * dys;
        }
      }
    }
    for (int i = H - 1; i >= 0; --i) {
      constexpr int NW = MT * (TC::NK0 > MT ? TC::NK0 : MT);
      f4 oldw[NW];
      if (i == 0) {
        if (R0 < MT) load_tiles(TC::tile_l0(R0, 0), (MT - R0) * TC::NK0, oldw + R0 * TC::NK0);
      } else {
        if (!kResident0 || i != H - 1) load_tiles(TC::tile_h(H, i, 0, 0), MT * MT, oldw);
      }
      const float* ai = abuf + i * S * AS;
      // delta_i = d L / d x_i = (d L / d h_i) * act'(x_i), x = W h + b in
      // world units (a_i holds x / (2 pi) for the periodic activations)
      f4 dbias[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) dbias[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int t = 0; t < NTC; ++t)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const f4 a = *reinterpret_cast<const f4*>(ai + (16 * t + nn) * AS + 16 * mt + 4 * g);
          f4 da;
#pragma unroll
          for (int j = 0; j < 4; ++j) da[j] = dh[t][mt][j] * act_d<ACT>(a[j]);
          dh[t][mt] = da;
          *reinterpret_cast<f4*>(dbuf + (16 * t + nn) * AS + 16 * mt + 4 * g) = da;
          dbias[mt] += da;
        }
      if (i >= 1) {
        // bias gradient: this lane's samples, summed over the row's 16 points
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const f4 sum = row16_sum(dbias[mt]);
          if (nn == 0) bacc[((i - 1) * MT + mt) * 4 + g] += sum;
        }
      }
      wave_lds_sync();
      // dW_i = delta_i h_i^T over the chunk's samples
      if (i == 0) {
#pragma unroll
        for (int mo = 0; mo < MT; ++mo)
#pragma unroll
          for (int nk = 0; nk < TC::NK0; ++nk) {
            f4 dw = {0.0f, 0.0f, 0.0f, 0.0f};
            const int col = 16 * nk + nn;
#pragma unroll
            for (int q = 0; q < S / 4; ++q) {
              const int s = 4 * q + g;
              const float a = dbuf[s * AS + 16 * mo + nn];
              const float b = col < G::KROW ? feat[s * G::ROW + col] : 0.0f;
              dw = PR::mma(a, b, dw);
            }
            if (mo < R0) {
              acc0[mo * TC::NK0 + nk] += dw;
            } else {
              put_tile(TC::tile_l0(mo, nk), oldw[mo * TC::NK0 + nk], dw);
            }
          }
      } else {
        const float* ap = abuf + (i - 1) * S * AS;
#pragma unroll
        for (int mo = 0; mo < MT; ++mo)
#pragma unroll
          for (int nk = 0; nk < MT; ++nk) {
            f4 dw = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int q = 0; q < S / 4; ++q) {
              const int s = 4 * q + g;
              const float a = dbuf[s * AS + 16 * mo + nn];
              const float b = act_el<ACT, false>(ap[s * AS + 16 * nk + nn], value_role());
              dw = PR::mma(a, b, dw);
            }
            if (kResident0 && i == H - 1) {
              accH[mo * MT + nk] += dw;
            } else {
              put_tile(TC::tile_h(H, i, mo, nk), oldw[mo * MT + nk], dw);
            }
          }
      }
      if (i >= 1) {
        // d L / d h_{i-1} = W_i^T delta_i (MFMA, B = delta in D layout)
        const float* WH = reinterpret_cast<const float*>(smem + G::W0A + (i - 1) * G::HID);
        const float* WB = reinterpret_cast<const float*>(back + (i - 1) * TC::WB);
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
          f4 nd2[MT];
#pragma unroll
          for (int mk = 0; mk < MT; ++mk) nd2[mk] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int q = 0; q < 4 * MT; ++q) {
            if constexpr (TC::kBackCopy) {
              const float b = dh[t][q / 4][q % 4];
#pragma unroll
              for (int mk = 0; mk < MT; ++mk) nd2[mk] = PR::mma(WB[(mk * 4 * MT + q) * kWave + lane], b, nd2[mk]);
            } else {
              const float b = dh[t][q / 4][q % 4] * inv_sc;
#pragma unroll
              for (int mk = 0; mk < MT; ++mk)
                nd2[mk] = PR::mma(WH[((q / 4) * 4 * MT + 4 * mk) * kWave + (q % 4) + wt_lane], b, nd2[mk]);
            }
          }
#pragma unroll
          for (int mk = 0; mk < MT; ++mk) dh[t][mk] = nd2[mk];
        }
      } else {
        // d L / d z = W_0[:, latent]^T delta_0 -> zbuf[s][f]
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
          f4 dz = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int q = 0; q < 4 * MT; ++q) {
            if constexpr (TC::kBackCopy) {
              const float* WZ = reinterpret_cast<const float*>(back + (H - 1) * TC::WB);
              dz = PR::mma(WZ[q * kWave + lane], dh[t][q / 4][q % 4], dz);
            } else {
              const float a = nn < F ? W0[(q / 4) * G::Q0 * kWave + (q % 4) + wz_lane] : 0.0f;
              dz = PR::mma(a, dh[t][q / 4][q % 4] * inv_sc, dz);
            }
          }
          if (4 * g < F) *reinterpret_cast<f4*>(zbuf + (16 * t + nn) * TC::ZS + 4 * g) = dz;
        }
      }
      wave_lds_sync();
    }
    // ---------------- dL/dz and the latent cell of this lane's point
    if (ok) {
      int ix, iy, iz;
      float fx, fy, fz;
      axis_cell(px, nd.R, ix, fx);
      axis_cell(py, nd.R, iy, fy);
      axis_cell(pz, nd.R, iz, fz);
      const int cell = (iz * (nd.R - 1) + iy) * (nd.R - 1) + ix;
      cell_out[idx] = cell;
      rank_out[idx] = atomicAdd(cell_count + cell, 1);
      float4* dst = reinterpret_cast<float4*>(dz_out + idx * F);
#pragma unroll
      for (int q = 0; q < F / 4; ++q)
        dst[q] = make_float4(zbuf[lane * TC::ZS + 4 * q], zbuf[lane * TC::ZS + 4 * q + 1],
                             zbuf[lane * TC::ZS + 4 * q + 2], zbuf[lane * TC::ZS + 4 * q + 3]);
    }
    first = false;
  }
#pragma unroll
  for (int k = 0; k < NR0; ++k)
    reinterpret_cast<f4*>(slice + TC::tile_l0(k / TC::NK0, k % TC::NK0) * 256)[lane] = acc0[k];
  if constexpr (kResident0) {
    if (H >= 2) {
#pragma unroll
      for (int k = 0; k < MT * MT; ++k)
        reinterpret_cast<f4*>(slice + TC::tile_h(H, H - 1, k / MT, k % MT) * 256)[lane] = accH[k];
    }
  }
#pragma unroll
  for (int k = 0; k < MT; ++k) reinterpret_cast<f4*>(slice + TC::tile_out(H, k) * 256)[lane] = accO[k];
  // the bias sums into the slice's per-lane partial layout: lane 16 g holds
  // row group g's sums, the row's other lanes zero
  for (int i = 1; i < H; ++i)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const f4 b = bacc[((i - 1) * MT + mt) * 4 + g];
      const f4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
      reinterpret_cast<f4*>(slice + TC::tile_bias(H, i, mt) * 256)[lane] = nn == 0 ? b : zero4;
    }
  // ---------------- per-wave partials of the output biases and the loss
#pragma unroll
  for (int o = 0; o < 4; ++o) slice[TC::tiles(H) * 256 + 64 * o + lane] = dbo_acc[o];
  slice[TC::tiles(H) * 256 + 256 + lane] = loss_acc;
}

// ------------------------------------------------- FP16-MFMA training
//
// The same step with the network in FP16 on the 16x16x32 and 16x16x16 MFMA
// with FP32 accumulation: the forward pass is the FP16 render's (its staged
// weight fragments and input rows, activations handed from layer to layer
// as D -> B fragments), the backward pass runs W^T on FP16 fragments of the
// unscaled master weights, and every weight-gradient tile is an FP16 GEMM
// over the chunk's 16 points. The parameters, the gradients they receive,
// the latent gather and Adam stay FP32, and the slice layout is the FP32
// step's, so the reduction kernels are shared.
//
// FP16 holds the output gradient only if it is scaled: dL/dy of the mean L1
// loss is sign / n, far below FP16's normal range for 2^18 points. The kernel
// multiplies dL/dy by gs = 2^floor(log2 n) (dscale = gs / n in [0.5, 1]) and
// every gradient it writes by 1 / gs, a power of two, so the scaling itself
// is exact.
template <int C, int F, int L, int ACT>
struct TrainCfgH {
  using T32 = TrainCfg<C, F, L, ACT>;  // slice layout shared with the FP32 step
  using CF = Cfg<kF16, C, F, L, ACT, 0>;
  using G = typename CF::G;
  static constexpr int S = 16;  // points per wave chunk (one N-tile)
  static constexpr int MT = G::MT;
  // The input-row columns must tile as in the FP32 layout (latent, Fourier
  // and the x y z 1 tail at the same columns; FP16's extra pad is zero).
  static_assert(G::KMAIN == T32::G::KMAIN && (G::KROW + 15) / 16 == T32::NK0, "row layouts differ");
  // [channel][point] FP16 buffers: 20 halves per channel row, so that the
  // 8-byte reads of 16 consecutive channel rows at one point offset fall on
  // distinct banks
  static constexpr int HSTR = 20;
  static constexpr int FEAT = S * G::ROW_DW * 4;
  static constexpr int CH = C * HSTR * 2;
  static constexpr int ACTD = MT * kWave * 8;  // one layer's act' (4 halves per lane and M-tile)
  static constexpr int DY = 64 * 4;
  static constexpr int ZS = 20;
  static constexpr int ZBUF = S * ZS * 4;
  static constexpr int BACC = MT * 4 * 16;     // one layer's bias sums: [M-tile][row group] f4
  __host__ __device__ static int wave_bytes(int H) { return FEAT + H * CH + H * ACTD + CH + DY + ZBUF + (H - 1) * BACC; }
  // transposed fragments: W_i^T (i = 1..H-1) and W_0's latent columns
  static constexpr int WBA = MT * G::HS32 * kWave * 16;
  static constexpr int WB = WBA + MT * G::HS16 * kWave * 8;
  static constexpr int WZA = G::HS32 * kWave * 16;
  static constexpr int WZ = WZA + G::HS16 * kWave * 8;
  __host__ __device__ static int back_bytes(int H) { return (H - 1) * WB + WZ; }
  __host__ __device__ static int block_bytes(int H, int waves) {
    return G::weight_bytes(H) + back_bytes(H) + waves * wave_bytes(H);
  }
};

// FP16 A fragments of the transposed layers. Row r of M-tile mk is input
// channel 16 mk + r; the K slots follow the order in which the forward pass
// packs a D fragment into a B fragment (slot j of lane group g in K32 step s
// is channel 32 s + 4 g + j for j < 4, 32 s + 16 + 4 g + j - 4 otherwise; the
// K16 step of c = 48 holds channels 32 + 4 g + j), so that a delta in D
// layout, packed the same way, is the B operand. Unscaled master weights:
// the deltas are in world units.
template <class TH>
__device__ void stage_backward_h(const NetDev& nd, char* p) {
  using G = typename TH::G;
  constexpr int C = TH::CF::C, F = TH::CF::F, MT = TH::MT;
  const int H = nd.H, K0 = G::K0IN;
  const float* w = nd.weights;
  const int tid = threadIdx.x, nt = blockDim.x;
  auto stage = [&](char* dst, int mtiles, auto val) {  // val(row channel, K channel)
    _Float16* A = reinterpret_cast<_Float16*>(dst);
    for (int e = tid; e < mtiles * G::HS32 * kWave * 8; e += nt) {
      const int j = e & 7, lane = (e >> 3) & 63, s = (e >> 9) % G::HS32, mk = (e >> 9) / G::HS32;
      const int g = lane >> 4;
      const int o = 32 * s + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
      A[e] = (_Float16)val(16 * mk + (lane & 15), o);
    }
    if constexpr (G::HS16 > 0) {
      _Float16* T = reinterpret_cast<_Float16*>(dst + mtiles * G::HS32 * kWave * 16);
      for (int e = tid; e < mtiles * kWave * 4; e += nt) {
        const int j = e & 3, lane = (e >> 2) & 63, mk = e >> 8;
        T[e] = (_Float16)val(16 * mk + (lane & 15), 16 * (MT - 1) + 4 * (lane >> 4) + j);
      }
    }
  };
  for (int i = 1; i < H; ++i) {
    const float* Wi = w + (long long)C * K0 + C + (long long)(i - 1) * (C * C + C);
    stage(p + (i - 1) * TH::WB, MT, [&](int k, int o) { return Wi[o * C + k]; });
  }
  stage(p + (H - 1) * TH::WB, 1, [&](int m, int o) { return m < F ? w[(long long)o * K0 + 3 + m] : 0.0f; });
}

template <int C, int F, int L, int ACT>
__global__ __launch_bounds__(kTrainWavesPerBlock * 64) void fwd_bwd_h_kernel(
    NetDev nd, KeyTimes kt, const float* xyz, const float* times, long long n, const float* target,
    const float* target_grad, float gw3, float* dz_out, int* cell_out, int* cell_count, int* rank_out, float* ws,
    int n_waves, float dscale, float inv_gs) {
  using TH = TrainCfgH<C, F, L, ACT>;
  using T32 = typename TH::T32;
  using CF = typename TH::CF;
  using G = typename TH::G;
  using PR = PrecT<kF16>;
  using VA = typename PR::VA;
  using VT = typename PR::VT;
  using E = _Float16;
  constexpr int MT = TH::MT, S = TH::S, HSTR = TH::HSTR, HS32 = G::HS32, HS16 = G::HS16;
  const int H = nd.H, NO = nd.NO;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  stage_weights<CF>(nd, smem);
  char* back = smem + G::weight_bytes(H);
  stage_backward_h<TH>(nd, back);
  __syncthreads();
  const int wave_l = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + wave_l;
  if (wave >= n_waves) return;
  const int g = lane >> 4, nn = lane & 15;
  char* wbase = back + TH::back_bytes(H) + wave_l * TH::wave_bytes(H);
  E* feat = reinterpret_cast<E*>(wbase);
  E* hbuf = reinterpret_cast<E*>(wbase + TH::FEAT);  // h_i = act(a_i): [layer][channel][point]
  char* actd = wbase + TH::FEAT + H * TH::CH;          // act'(a_i): [layer][M-tile][lane] x 4
  E* dbuf = reinterpret_cast<E*>(actd + H * TH::ACTD);  // delta_i: [channel][point]
  float* dy = reinterpret_cast<float*>(reinterpret_cast<char*>(dbuf) + TH::CH);
  float* zbuf = dy + 64;
  // hidden layers' bias gradients over the wave's chunks (see fwd_bwd_kernel)
  f4* bacc = reinterpret_cast<f4*>(reinterpret_cast<char*>(zbuf) + TH::ZBUF);
  for (int e = lane; e < (H - 1) * MT * 4; e += kWave) bacc[e] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  float* slice = ws + (size_t)wave * T32::slice(H);
  const VA* W0A = reinterpret_cast<const VA*>(smem);
  const VA* W0T = reinterpret_cast<const VA*>(smem + G::W0A);
  const char* wout_p = smem + G::W0A + G::W0T + (H - 1) * G::HID;
  const f4 b_out = *reinterpret_cast<const f4*>(wout_p + G::WOA + G::WOT);
  const float* w_out = nd.weights + (long long)C * G::K0IN + C + (long long)(H - 1) * (C * C + C);
  const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  float loss_acc = 0.0f;
  f4 dbo_acc = zero;
  const long long nchunks = (n + S - 1) / S;
  bool first = true;
  // Slice updates: a layer's running tile sums are loaded together before
  // its gradient MFMAs (the loads are in flight meanwhile), then each sum is
  // stored branch-free from a VALU select (see fwd_bwd_kernel); the first
  // chunk's loads read stale workspace and are discarded by the select.
  auto load_tiles = [&](int t0, int cnt, f4* old) {
    for (int k = 0; k < cnt; ++k) old[k] = reinterpret_cast<const f4*>(slice + (t0 + k) * 256)[lane];
  };
  auto put_tile = [&](int tile, f4 old, f4 v) {
    f4 r;
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = first ? v[j] : old[j] + v[j];
    reinterpret_cast<f4*>(slice + tile * 256)[lane] = r;
  };
  // positions, times and targets one chunk ahead (see fwd_bwd_kernel)
  float npx, npy, npz, npt, ntg;
  auto load_point = [&](long long cc) {
    const long long j = cc * S + lane;
    npx = npy = npz = npt = ntg = 0.0f;
    if (lane < S && cc < nchunks && j < n) {
      npx = xyz[3 * j];
      npy = xyz[3 * j + 1];
      npz = xyz[3 * j + 2];
      if (times) npt = times[j];
      ntg = target[j];
    }
  };
  // layer-0 and the last two hidden layers' weight-gradient tiles in
  // registers for c = 32, the output layer's at every width (see
  // fwd_bwd_kernel, which keeps one hidden layer's: a second spills there)
  constexpr bool kResident0 = C == 32;
  constexpr int R0 = kResident0 ? MT : 1;  // layer-0 M-tiles held (the first one at c = 48)
  constexpr int NR0 = R0 * T32::NK0, NRO = MT, NRH = kResident0 ? MT * MT : 1;
  f4 acc0[NR0], accO[NRO], accH[NRH], accH2[NRH];
#pragma unroll
  for (int k = 0; k < NR0; ++k) acc0[k] = zero;
#pragma unroll
  for (int k = 0; k < NRO; ++k) accO[k] = zero;
#pragma unroll
  for (int k = 0; k < NRH; ++k) accH[k] = accH2[k] = zero;
  load_point(wave);
  for (long long c = wave; c < nchunks; c += n_waves) {
    const long long idx = c * S + lane;
    const bool ok = lane < S && idx < n;
    const float px = npx, py = npy, pz = npz, pt = npt, tg = ntg;
    {
      // quad lane >> 2 builds that point's row (see fwd_bwd_kernel)
      const int src = lane >> 2;
      const float qx = __shfl(px, src, 64), qy = __shfl(py, src, 64), qz = __shfl(pz, src, 64);
      if (nd.K == 1) {
        write_row_quad<CF>(feat + src * G::ROW, make_latent_src(nd, 0, 0.0f), lane & 3, qx, qy, qz);
      } else {
        int key;
        float kw;
        key_pair(kt, nd.K, __shfl(pt, src, 64), key, kw);
        write_row_quad<CF>(feat + src * G::ROW, make_latent_src(nd, key, kw), lane & 3, qx, qy, qz);
      }
    }
    wave_lds_sync();
    load_point(c + n_waves);
    // ---------------- forward (FP16 MFMA); keep act'(a_i) and h_i
    f4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = zero;
#pragma unroll
    for (int s = 0; s < G::S0; ++s) {
      const VA b = *reinterpret_cast<const VA*>(feat + nn * G::ROW + 32 * s + 8 * g);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = PR::mma(W0A[(mt * G::S0 + s) * kWave + lane], b, acc[mt]);
    }
    {
      const VA b = *reinterpret_cast<const VA*>(feat + nn * G::ROW + G::KMAIN + 8 * (g % (G::KT / 8)));
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = PR::mma(W0T[mt * kWave + lane], b, acc[mt]);
    }
    VA bA[HS32];
    VT bT;
    const char* p = smem + G::W0A + G::W0T;
    for (int i = 0; i < H; ++i) {
      E* hb = hbuf + i * C * HSTR;
      h4* ad = reinterpret_cast<h4*>(actd + i * TH::ACTD);
      float hv[MT][4];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        h4 dv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float a = acc[mt][j];
          hv[mt][j] = act_el<ACT, false>(a, value_role());
          dv[j] = (E)act_d<ACT>(a);
          hb[(16 * mt + 4 * g + j) * HSTR + nn] = (E)hv[mt][j];
        }
        ad[mt * kWave + lane] = dv;
      }
#pragma unroll
      for (int s = 0; s < HS32; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bA[s][j] = (E)hv[2 * s][j];
          bA[s][j + 4] = (E)hv[2 * s + 1][j];
        }
      if constexpr (HS16 > 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) bT[j] = (E)hv[MT - 1][j];
      }
      if (i + 1 < H) {
        const VA* WA = reinterpret_cast<const VA*>(p);
        const VT* WT = reinterpret_cast<const VT*>(p + G::WHA);
        const float* BHp = reinterpret_cast<const float*>(p + G::WHA + G::WHT);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          acc[mt] = *reinterpret_cast<const f4*>(BHp + 16 * mt + 4 * g);
#pragma unroll
          for (int s = 0; s < HS32; ++s) acc[mt] = PR::mma(WA[(mt * HS32 + s) * kWave + lane], bA[s], acc[mt]);
          if constexpr (HS16 > 0) acc[mt] += PR::mmt(WT[mt * kWave + lane], bT, zero);
        }
        p += G::HID;
      }
    }
    // output layer: N-tile 0's weights sit in rows 0..3, so lanes < 16 hold
    // their own point's outputs
    f4 out = zero;
#pragma unroll
    for (int s = 0; s < HS32; ++s) out = PR::mma(reinterpret_cast<const VA*>(p)[s * kWave + lane], bA[s], out);
    if constexpr (HS16 > 0) out += PR::mmt(reinterpret_cast<const VT*>(p + G::WOA)[lane], bT, zero);
    // ---------------- loss and the scaled dL/dy of this lane's own point
    const f4 yv = out + b_out;
    const float d = sigmoid_f(yv[0]);
    float gy = 0.0f;
    f4 dyo = zero;
    if (ok) {
      const float r = d - tg;
      loss_acc += fabsf(r);
      gy = (r > 0.0f ? 1.0f : (r < 0.0f ? -1.0f : 0.0f)) * dscale;
      if (target_grad) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float rg = yv[1 + a] - target_grad[3 * idx + a];
          loss_acc += gw3 * fabsf(rg);
          dyo[1 + a] = (rg > 0.0f ? gw3 : (rg < 0.0f ? -gw3 : 0.0f)) * dscale;
        }
      }
    }
    dyo[0] = gy * d * (1.0f - d);
    dbo_acc += dyo;
    if (lane < S) {
#pragma unroll
      for (int o = 0; o < 4; ++o) dy[o * S + lane] = dyo[o];
    }
    wave_lds_sync();
    // ---------------- output weights: dW_H[o][k] = sum_s dy[o][s] h_{H-1}[k][s]
    {
      const E* hl = hbuf + (H - 1) * C * HSTR;
      VT ay;
#pragma unroll
      for (int j = 0; j < 4; ++j) ay[j] = nn < NO ? (E)dy[nn * S + 4 * g + j] : (E)0.0f;
#pragma unroll
      for (int nk = 0; nk < MT; ++nk) {
        const VT b = *reinterpret_cast<const VT*>(hl + (16 * nk + nn) * HSTR + 4 * g);
        accO[nk] += PR::mmt(ay, b, zero) * inv_gs;
      }
    }
    // ---------------- backward
    f4 dh[MT];  // d L / d h_i, D layout
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) dh[mt] = zero;
    for (int o = 0; o < NO; ++o) {
      const float dys = dy[o * S + nn];
      const float* wr = w_out + o * C;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const f4 wo = {wr[16 * mt + 4 * g + 0], wr[16 * mt + 4 * g + 1], wr[16 * mt + 4 * g + 2],
                       wr[16 * mt + 4 * g + 3]};
        dh[mt] += wo * dys;
      }
    }
    for (int i = H - 1; i >= 0; --i) {
      // this layer's running sums: dW_i, and for i >= 1 the bias partials
      constexpr int NW = MT * (T32::NK0 > MT ? T32::NK0 : MT);
      f4 oldw[NW];
      if (i == 0) {
        if (R0 < MT) load_tiles(T32::tile_l0(R0, 0), (MT - R0) * T32::NK0, oldw + R0 * T32::NK0);
      } else {
        if (!kResident0 || i < H - 2) load_tiles(T32::tile_h(H, i, 0, 0), MT * MT, oldw);
      }
      const h4* ad = reinterpret_cast<const h4*>(actd + i * TH::ACTD);
      // delta_i = (d L / d h_i) * act'(a_i), world units
      float dv[MT][4];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const h4 a = ad[mt * kWave + lane];
        f4 da;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          dv[mt][j] = dh[mt][j] * (float)a[j];
          da[j] = dv[mt][j];
          dbuf[(16 * mt + 4 * g + j) * HSTR + nn] = (E)dv[mt][j];
        }
        if (i >= 1) {
          const f4 sum = row16_sum(da * inv_gs);
          if (nn == 0) bacc[((i - 1) * MT + mt) * 4 + g] += sum;
        }
      }
      VA bD[HS32];
      VT bDT;
#pragma unroll
      for (int s = 0; s < HS32; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bD[s][j] = (E)dv[2 * s][j];
          bD[s][j + 4] = (E)dv[2 * s + 1][j];
        }
      if constexpr (HS16 > 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) bDT[j] = (E)dv[MT - 1][j];
      }
      wave_lds_sync();
      // dW_i = delta_i h_{i-1}^T over the chunk's points (16x16x16, K = points)
      if (i == 0) {
        // the input row: FP16 rows hold 2 cos in the cosine block (the
        // forward fragments carry half those weights), so that gradient
        // column is halved
#pragma unroll
        for (int nk = 0; nk < T32::NK0; ++nk) {
          const int col = 16 * nk + nn;
          VT b;
#pragma unroll
          for (int j = 0; j < 4; ++j) b[j] = col < G::KROW ? feat[(4 * g + j) * G::ROW + col] : (E)0.0f;
          const float cs = (col >= F + 3 * L && col < F + 6 * L) ? 0.5f * inv_gs : inv_gs;
#pragma unroll
          for (int mo = 0; mo < MT; ++mo) {
            const VT a = *reinterpret_cast<const VT*>(dbuf + (16 * mo + nn) * HSTR + 4 * g);
            if (mo < R0) {
              acc0[mo * T32::NK0 + nk] += PR::mmt(a, b, zero) * cs;
            } else {
              put_tile(T32::tile_l0(mo, nk), oldw[mo * T32::NK0 + nk], PR::mmt(a, b, zero) * cs);
            }
          }
        }
      } else {
        const E* hp = hbuf + (i - 1) * C * HSTR;
#pragma unroll
        for (int nk = 0; nk < MT; ++nk) {
          const VT b = *reinterpret_cast<const VT*>(hp + (16 * nk + nn) * HSTR + 4 * g);
#pragma unroll
          for (int mo = 0; mo < MT; ++mo) {
            const VT a = *reinterpret_cast<const VT*>(dbuf + (16 * mo + nn) * HSTR + 4 * g);
            if (kResident0 && i == H - 1) {
              accH[mo * MT + nk] += PR::mmt(a, b, zero) * inv_gs;
            } else if (kResident0 && i == H - 2) {
              accH2[mo * MT + nk] += PR::mmt(a, b, zero) * inv_gs;
            } else {
              put_tile(T32::tile_h(H, i, mo, nk), oldw[mo * MT + nk], PR::mmt(a, b, zero) * inv_gs);
            }
          }
        }
      }
      if (i >= 1) {
        // d L / d h_{i-1} = W_i^T delta_i
        const char* wb = back + (i - 1) * TH::WB;
        const VA* WBA = reinterpret_cast<const VA*>(wb);
        const VT* WBT = reinterpret_cast<const VT*>(wb + TH::WBA);
#pragma unroll
        for (int mk = 0; mk < MT; ++mk) {
          f4 a2 = zero;
#pragma unroll
          for (int s = 0; s < HS32; ++s) a2 = PR::mma(WBA[(mk * HS32 + s) * kWave + lane], bD[s], a2);
          if constexpr (HS16 > 0) a2 += PR::mmt(WBT[mk * kWave + lane], bDT, zero);
          dh[mk] = a2;
        }
      } else {
        // d L / d z = W_0[:, latent]^T delta_0 -> zbuf[point][channel]
        const char* wz = back + (H - 1) * TH::WB;
        f4 dz = zero;
#pragma unroll
        for (int s = 0; s < HS32; ++s) dz = PR::mma(reinterpret_cast<const VA*>(wz)[s * kWave + lane], bD[s], dz);
        if constexpr (HS16 > 0) dz += PR::mmt(reinterpret_cast<const VT*>(wz + TH::WZA)[lane], bDT, zero);
        if (4 * g < F) *reinterpret_cast<f4*>(zbuf + nn * TH::ZS + 4 * g) = dz * inv_gs;
      }
      wave_lds_sync();
    }
    // ---------------- dL/dz and the latent cell of this lane's point
    if (ok) {
      int ix, iy, iz;
      float fx, fy, fz;
      axis_cell(px, nd.R, ix, fx);
      axis_cell(py, nd.R, iy, fy);
      axis_cell(pz, nd.R, iz, fz);
      const int cell = (iz * (nd.R - 1) + iy) * (nd.R - 1) + ix;
      cell_out[idx] = cell;
      rank_out[idx] = atomicAdd(cell_count + cell, 1);
      float4* dst = reinterpret_cast<float4*>(dz_out + idx * F);
#pragma unroll
      for (int q = 0; q < F / 4; ++q)
        dst[q] = make_float4(zbuf[lane * TH::ZS + 4 * q], zbuf[lane * TH::ZS + 4 * q + 1],
                             zbuf[lane * TH::ZS + 4 * q + 2], zbuf[lane * TH::ZS + 4 * q + 3]);
    }
    first = false;
  }
#pragma unroll
  for (int k = 0; k < NR0; ++k)
    reinterpret_cast<f4*>(slice + T32::tile_l0(k / T32::NK0, k % T32::NK0) * 256)[lane] = acc0[k];
  if constexpr (kResident0) {
    if (H >= 2) {
#pragma unroll
      for (int k = 0; k < MT * MT; ++k)
        reinterpret_cast<f4*>(slice + T32::tile_h(H, H - 1, k / MT, k % MT) * 256)[lane] = accH[k];
    }
    if (H >= 3) {
#pragma unroll
      for (int k = 0; k < MT * MT; ++k)
        reinterpret_cast<f4*>(slice + T32::tile_h(H, H - 2, k / MT, k % MT) * 256)[lane] = accH2[k];
    }
  }
#pragma unroll
  for (int k = 0; k < MT; ++k) reinterpret_cast<f4*>(slice + T32::tile_out(H, k) * 256)[lane] = accO[k];
  for (int i = 1; i < H; ++i)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const f4 b = bacc[((i - 1) * MT + mt) * 4 + g];
      reinterpret_cast<f4*>(slice + T32::tile_bias(H, i, mt) * 256)[lane] = nn == 0 ? b : zero;
    }
  dbo_acc *= inv_gs;
#pragma unroll
  for (int o = 0; o < 4; ++o) slice[T32::tiles(H) * 256 + 64 * o + lane] = dbo_acc[o];
  slice[T32::tiles(H) * 256 + 256 + lane] = loss_acc;
}

// Sums the wave slices in a fixed order into the packed gradient, in two
// stages so that the reads are coalesced and plenty of them are in flight:
// slice_sum_kernel adds groups of kGroup consecutive slices element-wise
// (partial[g][e], threads along e), gather_kernel then locates every weight's
// terms in the slice layout and adds them over the groups. Both orders are
// fixed, so the result is bitwise reproducible.
constexpr int kGroup = 256;

__global__ void slice_sum_kernel(const float* ws, int n_waves, int sl, float* partial) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (e >= sl) return;
  const int w0 = g * kGroup, w1 = min(w0 + kGroup, n_waves);
  // eight independent partial sums keep eight loads in flight; they are
  // combined in a fixed order
  float s8[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  int w = w0;
  for (; w + 8 <= w1; w += 8)
#pragma unroll
    for (int k = 0; k < 8; ++k) s8[k] += ws[(size_t)(w + k) * sl + e];
  for (; w < w1; ++w) s8[0] += ws[(size_t)w * sl + e];
  partial[(size_t)g * sl + e] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
}

template <int C, int F, int L, int ACT, int TE, int FM>
__global__ void gather_kernel(int H, int NO, const float* partial, int n_groups, float* d_weights, float* out_loss,
                              float loss_scale) {
  using TC = TrainCfg<C, F, L, ACT, TE, FM>;
  using G = typename TC::G;
  const int K0 = G::K0IN;
  const long long nw = (long long)C * K0 + C + (long long)(H - 1) * (C * C + C) + (long long)NO * (C + 1);
  const int SL = TC::slice(H);
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < nw + 1;
       j += (long long)gridDim.x * blockDim.x) {
    // locate weight j: a list of (offset within slice) terms to add
    int base = -1, count = 0, stride = 0;
    if (j == nw) {  // loss
      base = TC::tiles(H) * 256 + 256;
      count = 64;
      stride = 1;
    } else {
      long long r = j;
      const long long l0 = (long long)C * K0;
      if (r < l0 + C) {
        int o, col;
        if (r < l0) {
          o = (int)(r / K0);
          const int k = (int)(r % K0);
          col = G::feat_col(k);
        } else {
          o = (int)(r - l0);
          col = G::KMAIN + 3;
        }
        const int tile = TC::tile_l0(o / 16, col / 16);
        base = tile * 256 + (16 * ((o % 16) / 4) + col % 16) * 4 + o % 4;
        count = 1;
      } else {
        r -= l0 + C;
        const long long per = (long long)C * C + C;
        const int i = 1 + (int)(r / per);
        if (i < H) {
          r %= per;
          if (r < (long long)C * C) {
            const int o = (int)(r / C), k = (int)(r % C);
            base = TC::tile_h(H, i, o / 16, k / 16) * 256 + (16 * ((o % 16) / 4) + k % 16) * 4 + o % 4;
            count = 1;
          } else {
            const int o = (int)(r - (long long)C * C);
            base = TC::tile_bias(H, i, o / 16) * 256 + (16 * ((o % 16) / 4)) * 4 + o % 4;
            count = 16;
            stride = 4;
          }
        } else {
          r -= (long long)(H - 1) * per;
          if (r < (long long)NO * C) {
            // W_out[o][k]: row o of the output tile, held by lane k % 16
            const int o = (int)(r / C), k = (int)(r % C);
            base = TC::tile_out(H, k / 16) * 256 + (k % 16) * 4 + o;
            count = 1;
          } else {
            base = TC::tiles(H) * 256 + 64 * (int)(r - (long long)NO * C);
            count = 64;
            stride = 1;
          }
        }
      }
    }
    // sums of 16 or 64 terms per group (the hidden and output biases, the
    // loss) are gather_long_kernel's
    if (count > 1) continue;
    // sequential adds in a fixed order
    float s = 0.0f;
    for (int g = 0; g < n_groups; ++g) {
      const float* pg = partial + (size_t)g * SL + base;
#pragma unroll 8
      for (int c = 0; c < count; ++c) s += pg[c * stride];
    }
    if (j == nw) {
      if (out_loss) *out_loss = s * loss_scale;
    } else {
      d_weights[j] = s;
    }
  }
}

// The weights whose gradient sums many partials per group, one wave each:
// the hidden-layer biases (16 lane partials per group), the output biases and
// the loss (64). Lane l adds its term over the groups in order, then the wave
// adds the lanes in a fixed butterfly, so the result is bitwise reproducible.
template <int C, int F, int L, int ACT, int TE, int FM>
__global__ __launch_bounds__(64) void gather_long_kernel(int H, int NO, const float* partial, int n_groups,
                                                          float* d_weights, float* out_loss, float loss_scale) {
  using TC = TrainCfg<C, F, L, ACT, TE, FM>;
  using G = typename TC::G;
  const int e = blockIdx.x, lane = threadIdx.x;
  const int SL = TC::slice(H);
  const long long first_bias = (long long)C * G::K0IN + C;  // W_1 in the packed weights
  const long long per = (long long)C * C + C;
  int base, count, stride;
  long long j;  // destination weight (-1: the loss)
  if (e < (H - 1) * C) {
    const int i = 1 + e / C, o = e % C;
    j = first_bias + (long long)(i - 1) * per + (long long)C * C + o;
    base = TC::tile_bias(H, i, o / 16) * 256 + (16 * ((o % 16) / 4)) * 4 + o % 4;
    count = 16;
    stride = 4;
  } else if (e < (H - 1) * C + NO) {
    const int o = e - (H - 1) * C;
    j = first_bias + (long long)(H - 1) * per + (long long)NO * C + o;
    base = TC::tiles(H) * 256 + 64 * o;
    count = 64;
    stride = 1;
  } else {
    j = -1;
    base = TC::tiles(H) * 256 + 256;
    count = 64;
    stride = 1;
  }
  float a = 0.0f;
  if (lane < count)
    for (int g = 0; g < n_groups; ++g) a += partial[(size_t)g * SL + base + lane * stride];
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if (lane == 0) {
    if (j < 0) {
      if (out_loss) *out_loss = a * loss_scale;
    } else {
      d_weights[j] = a;
    }
  }
}

__global__ void fill_kernel(float* p, long long n, float v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Bias-corrected Adam (PyTorch's form): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr / bc1 * m / (sqrt(v) / sqrt(bc2) + eps).
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, long long n, float lr_bc1, float b1,
                            float b2, float inv_sqrt_bc2, float eps) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr_bc1 * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
  }
}

// ------------------------------------------ latent gradient by gathering

// Exclusive prefix sums of the per-cell point counts, off[c] = first sorted
// position of cell c, off[ncell] = n, cursor (when given) a copy of off: blocks of
// kCellBlock consecutive cells are summed (cell_block_sum_kernel), the block
// sums scanned by one workgroup (cell_block_scan_kernel), then every block
// scans its own cells from its block's offset (cell_scan_kernel).
constexpr int kCellThreads = 256, kCellItems = 16, kCellBlock = kCellThreads * kCellItems;

int cell_blocks(long long ncell) { return (int)((ncell + kCellBlock - 1) / kCellBlock); }

// Exclusive scan of v over the workgroup; *total receives the sum. wsum:
// LDS of one int per wave. Every thread of the workgroup must call it.
template <int kThreads>
__device__ inline int block_exclusive_scan(int v, int* wsum, int* total) {
  constexpr int kWaves = kThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const int t = wsum[w];
    before += w < wave ? t : 0;
    tot += t;
  }
  __syncthreads();  // wsum may be rewritten by the next call
  *total = tot;
  return before + incl - v;
}

__global__ __launch_bounds__(kCellThreads) void cell_block_sum_kernel(const int* count, int ncell, int* bsum) {
  __shared__ int wsum[kCellThreads / 64];
  const int b0 = blockIdx.x * kCellBlock;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kCellItems; ++k) {  // striped: coalesced
    const int c = b0 + k * kCellThreads + threadIdx.x;
    s += c < ncell ? count[c] : 0;
  }
  int total;
  (void)block_exclusive_scan<kCellThreads>(s, wsum, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the nb block sums in place; off[ncell]
// receives the grand total.
constexpr int kBlockScanThreads = 1024, kBlockScanItems = 8;
__global__ __launch_bounds__(kBlockScanThreads) void cell_block_scan_kernel(int* bsum, int nb, int* off_end) {
  __shared__ int wsum[kBlockScanThreads / 64];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kBlockScanThreads * kBlockScanItems) {
    const int base = c0 + threadIdx.x * kBlockScanItems;
    int x[kBlockScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kBlockScanItems; ++k) {
      x[k] = base + k < nb ? bsum[base + k] : 0;
      sum += x[k];
    }
    int total;
    int run = carry + block_exclusive_scan<kBlockScanThreads>(sum, wsum, &total);
#pragma unroll
    for (int k = 0; k < kBlockScanItems; ++k) {
      if (base + k < nb) bsum[base + k] = run;
      run += x[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) *off_end = carry;
}

// Block b: its cells' exclusive prefix sums from its block offset (bsum,
// or 0 when bsum is null); each thread takes kCellItems consecutive cells.
// With a single block (off_end set) the kernel also writes the total.
__global__ __launch_bounds__(kCellThreads) void cell_scan_kernel(const int* count, int ncell, const int* bsum, int* off,
                                                                 int* cursor, int* off_end) {
  __shared__ int wsum[kCellThreads / 64];
  const int base = blockIdx.x * kCellBlock + threadIdx.x * kCellItems;
  int x[kCellItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kCellItems; ++k) {
    x[k] = base + k < ncell ? count[base + k] : 0;
    sum += x[k];
  }
  int total;
  int run = (bsum ? bsum[blockIdx.x] : 0) + block_exclusive_scan<kCellThreads>(sum, wsum, &total);
#pragma unroll
  for (int k = 0; k < kCellItems; ++k) {
    if (base + k < ncell) {
      off[base + k] = run;
      if (cursor) cursor[base + k] = run;
    }
    run += x[k];
  }
  if (off_end && threadIdx.x == 0) *off_end = total;
}

// Counting sort: point i goes to the slot its cell count gave it when the
// forward-backward kernel counted it (its rank among the cell's points).
__global__ void bin_points_kernel(const int* cell, const int* rank, const int* off, long long n, int* order) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    order[off[cell[i]] + rank[i]] = (int)i;
}

// d_latent[k][v][f] = sum over the points p of the (up to) eight cells
// around vertex v of w_v(p) * b_k(p) * dz[p][f]: w_v the trilinear weight of
// v as a corner of p's cell, b_k the blend weight of keyframe k at p's time
// (Sec. 8; 1 for one keyframe). A group of 8 lpc consecutive threads shares a
// (keyframe, vertex): lpc threads per cell, each taking every lpc-th point
// of it (lpc = 1..8, a power of two, from the mean points per cell), and the
// group adds its sums with lane shuffles in a fixed order; every entry is
// written.
template <int F>
__global__ void latent_grad_kernel(const float* xyz, const float* times, KeyTimes kt, int K, int R,
                                   long long key_stride, const int* off, const int* order, const float* dz,
                                   float* d_latent, int lpc_log2) {
  const long long nv = (long long)R * R * R;
  const int lpc = 1 << lpc_log2, gsz = 8 << lpc_log2;
  const long long total = nv * K * gsz;  // a multiple of the group size: groups are active or idle as a whole
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int lig = (int)(t & (gsz - 1));
    const int b = lig >> lpc_log2, sub = lig & (lpc - 1);
    const long long kv = t >> (3 + lpc_log2);
    const int k = (int)(kv / nv);
    const long long v = kv % nv;
    const int vx = (int)(v % R), vy = (int)((v / R) % R), vz = (int)(v / ((long long)R * R));
    const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
    const int cx = vx - bx, cy = vy - by, cz = vz - bz;  // the cell with v as corner (bx, by, bz)
    float acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = 0.0f;
    if (cx >= 0 && cx <= R - 2 && cy >= 0 && cy <= R - 2 && cz >= 0 && cz <= R - 2) {
      const int c = (cz * (R - 1) + cy) * (R - 1) + cx;
      for (int s = off[c] + sub; s < off[c + 1]; s += lpc) {
        const int p = order[s];
        int ix, iy, iz;
        float fx, fy, fz;
        axis_cell(xyz[3 * p], R, ix, fx);
        axis_cell(xyz[3 * p + 1], R, iy, fy);
        axis_cell(xyz[3 * p + 2], R, iz, fz);
        float w = (bx ? fx : 1.0f - fx) * (by ? fy : 1.0f - fy) * (bz ? fz : 1.0f - fz);
        if (K > 1) {
          int key;
          float kw;
          key_pair(kt, K, times ? times[p] : 0.0f, key, kw);
          w *= (k == key ? 1.0f - kw : 0.0f) + (k == key + 1 ? kw : 0.0f);
        }
        const float4* src = reinterpret_cast<const float4*>(dz + (long long)p * F);
#pragma unroll
        for (int q = 0; q < F / 4; ++q) {
          const float4 d4 = src[q];
          acc[4 * q] = fmaf(w, d4.x, acc[4 * q]);
          acc[4 * q + 1] = fmaf(w, d4.y, acc[4 * q + 1]);
          acc[4 * q + 2] = fmaf(w, d4.z, acc[4 * q + 2]);
          acc[4 * q + 3] = fmaf(w, d4.w, acc[4 * q + 3]);
        }
      }
    }
    // sum over the group (fixed order: pairs, then quads, ...)
    for (int o = 1; o < gsz; o <<= 1)
#pragma unroll
      for (int f = 0; f < F; ++f) acc[f] += __shfl_xor(acc[f], o, 64);
    if (lig == 0) {
      float4* dst = reinterpret_cast<float4*>(d_latent + (long long)k * key_stride + v * F);
#pragma unroll
      for (int q = 0; q < F / 4; ++q) dst[q] = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
    }
  }
}

// FP16 training: no time inputs or Fourier matrix, and the FP16 input row
// must tile like the FP32 one (the four base shapes)
template <int C, int F, int L, int TE, int FM>
constexpr bool half_train_ok() {
  return TE == 0 && FM == 0 && Geo<kF16, C, F, L>::KMAIN == Geo<kF32, C, F, L>::KMAIN &&
         (Geo<kF16, C, F, L>::KROW + 15) / 16 == (Geo<kF32, C, F, L>::KROW + 15) / 16;
}

// The latent gradient in two passes, for a single keyframe:
// cell_partials_kernel sums, per cell, corner and point subset (points
// off[c] + sub, + 2^sub_log2, ...: 2^sub_log2 subsets keep dense cells'
// loops short), the trilinear-weighted dL/dz of the cell's points (each point
// read once, by the F/4 threads of its subset), and vertex_sum_kernel adds
// every vertex's cell-corner sums over its (up to) eight cells and their
// subsets in a fixed order. Against the one-pass gather (latent_grad_kernel),
// which reads each point once per vertex of its cell, this moves about a
// third of the bytes.
template <int F>
__global__ void cell_partials_kernel(const float* xyz, int R, long long ncell, int sub_log2, const int* off,
                                     const int* order, const float* dz, float* part) {
  constexpr int NQ = F / 4;
  const int nsub = 1 << sub_log2;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell * nsub * NQ;
       t += (long long)gridDim.x * blockDim.x) {
    const long long cs = t / NQ;  // cell * nsub + subset
    const long long c = cs >> sub_log2;
    const int sub = (int)(cs & (nsub - 1)), qd = (int)(t % NQ);
    f4 acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int s = off[c] + sub; s < off[c + 1]; s += nsub) {
      const int p = order[s];
      int ix, iy, iz;
      float fx, fy, fz;
      axis_cell(xyz[3 * p], R, ix, fx);
      axis_cell(xyz[3 * p + 1], R, iy, fy);
      axis_cell(xyz[3 * p + 2], R, iz, fz);
      const f4 d = reinterpret_cast<const f4*>(dz + (long long)p * F)[qd];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
        const float w = (bx ? fx : 1.0f - fx) * (by ? fy : 1.0f - fy) * (bz ? fz : 1.0f - fz);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[b][j] = fmaf(w, d[j], acc[b][j]);
      }
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) reinterpret_cast<f4*>(part + (((c * 8 + b) << sub_log2) + sub) * F)[qd] = acc[b];
  }
}

template <int F>
__global__ void vertex_sum_kernel(int R, int sub_log2, const float* part, float* d_latent) {
  constexpr int NQ = F / 4;
  const long long nv = (long long)R * R * R;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nv * NQ;
       t += (long long)gridDim.x * blockDim.x) {
    const long long v = t / NQ;
    const int qd = (int)(t % NQ);
    const int vx = (int)(v % R), vy = (int)((v / R) % R), vz = (int)(v / ((long long)R * R));
    f4 sum = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int cx = vx - (b & 1), cy = vy - ((b >> 1) & 1), cz = vz - (b >> 2);
      if (cx >= 0 && cx <= R - 2 && cy >= 0 && cy <= R - 2 && cz >= 0 && cz <= R - 2) {
        const long long c = ((long long)cz * (R - 1) + cy) * (R - 1) + cx;
        for (int sub = 0; sub < (1 << sub_log2); ++sub)
          sum += reinterpret_cast<const f4*>(part + (((c * 8 + b) << sub_log2) + sub) * F)[qd];
      }
    }
    reinterpret_cast<f4*>(d_latent + v * F)[qd] = sum;
  }
}

template <int C, int F, int L, int ACT, int TE = 0, int FM = 0>
struct TrainEntry {
  using TC = TrainCfg<C, F, L, ACT, TE, FM>;
  static int waves_per_block(int H) {
    const int fixed = TC::G::weight_bytes(H) + TC::back_bytes(H);
    int w = (160 * 1024 - fixed) / TC::wave_bytes(H);
    return w < 1 ? 0 : (w > kTrainWavesPerBlock ? kTrainWavesPerBlock : w);
  }
  template <class TH>
  static int waves_per_block_h(int H) {
    const int fixed = TH::G::weight_bytes(H) + TH::back_bytes(H);
    int w = (160 * 1024 - fixed) / TH::wave_bytes(H);
    return w < 1 ? 0 : (w > kTrainWavesPerBlock ? kTrainWavesPerBlock : w);
  }
  static int n_waves(long long n) {
    const long long c = (n + TC::S - 1) / TC::S;
    const long long cap = C == 48 ? kTrainMaxWaves48 : kTrainMaxWaves;
    return (int)(c < cap ? (c < 1 ? 1 : c) : cap);
  }
  static int n_groups(long long n) { return (n_waves(n) + kGroup - 1) / kGroup; }
  // wave slices, then the group partials of the reduction, then the per-point
  // dL/dz [n][F], cells [n], sorted order [n] and ranks within the cell [n],
  // and per cell the point counts and the offsets (+1)
  static size_t slices_bytes(const NetDev& nd, long long n) {
    return ((size_t)(n_waves(n) + n_groups(n)) * TC::slice(nd.H) * sizeof(float) + 15) / 16 * 16;
  }
  static size_t ws_bytes(const NetDev& nd, long long n) {
    const long long ncell = (long long)(nd.R - 1) * (nd.R - 1) * (nd.R - 1);
    return slices_bytes(nd, n) + (size_t)n * F * 4 + (size_t)n * 12 + (size_t)(2 * ncell + 1 + cell_blocks(ncell)) * 4;
  }
  static int run(const NetDev& nd, const KeyTimes& kt, float* latent, float* d_latent, float* d_weights,
                 const float* xyz, const float* times, long long n, const float* target,
                 const float* target_grad, float grad_weight, const float* dloss, float* out_loss, void* ws,
                 bool half, hipStream_t st) {
    const int H = nd.H;
    if (half && (!half_train_ok<C, F, L, TE, FM>() || !target)) return 1;
    const int wpb = waves_per_block(H);
    if (wpb < 1) return kLaunchNoLds;
    const int ncell = (nd.R - 1) * (nd.R - 1) * (nd.R - 1);
    char* wsb = (char*)ws + slices_bytes(nd, n);
    float* dz = (float*)wsb;
    int* cell = (int*)(wsb + (size_t)n * F * 4);
    int* order = cell + n;
    int* rank = order + n;
    int* count = rank + n;
    int* off = count + ncell;
    int* bsum = off + ncell + 1;  // cell_blocks(ncell) block sums
    hipLaunchKernelGGL(fill_kernel, dim3(grid_blocks(ncell, 256, device_cus() * 8)), dim3(256), 0, st, (float*)count,
                       (long long)ncell, 0.0f);  // zero bits: zero counts
    int rc = check_launch();
    if (rc) return rc;
    const int nw = n_waves(n);
    const size_t shm = (size_t)TC::block_bytes(H, wpb);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)fwd_bwd_kernel<C, F, L, ACT, TE, FM>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      attr = true;
    }
    NetDev nd2 = nd;
    nd2.latent = latent;
    nd2.grid_f16 = 0;
    if (n > 0 && half) {
      if constexpr (half_train_ok<C, F, L, TE, FM>()) {
        using TH = TrainCfgH<C, F, L, ACT>;
        const int wph = waves_per_block_h<TH>(H);
        if (wph < 1) return kLaunchNoLds;
        static bool attr_h = false;
        if (!attr_h) {
          (void)hipFuncSetAttribute((const void*)fwd_bwd_h_kernel<C, F, L, ACT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
          attr_h = true;
        }
        // dL/dy scaled by gs = 2^floor(log2 n) for FP16, gradients by 1 / gs
        const int e = std::ilogb((double)n);
        const double gs = std::ldexp(1.0, e);
        hipLaunchKernelGGL((fwd_bwd_h_kernel<C, F, L, ACT>), dim3((nw + wph - 1) / wph), dim3(wph * 64),
                           (size_t)TH::block_bytes(H, wph), st, nd2, kt, xyz, times, n, target, target_grad,
                           grad_weight / 3.0f, dz, cell, count, rank, (float*)ws, nw, (float)(gs / (double)n),
                           (float)(1.0 / gs));
        rc = check_launch();
        if (rc) return rc;
      }
    } else if (n > 0) {
      hipLaunchKernelGGL((fwd_bwd_kernel<C, F, L, ACT, TE, FM>), dim3((nw + wpb - 1) / wpb), dim3(wpb * 64), shm, st, nd2,
                         kt, xyz, times, n, target, target_grad, grad_weight / 3.0f, dloss, dz, cell, count, rank,
                         (float*)ws, nw, 1.0f / (float)n);
      rc = check_launch();
      if (rc) return rc;
    } else {
      // no points: every slice is zero
      hipLaunchKernelGGL(fill_kernel, dim3(grid_blocks((long long)nw * TC::slice(H), 256, device_cus() * 8)),
                         dim3(256), 0, st, (float*)ws, (long long)nw * TC::slice(H), 0.0f);
      rc = check_launch();
      if (rc) return rc;
    }
    // latent gradient: sort the points by cell, then gather per vertex
    const int nb = cell_blocks(ncell);
    if (nb > 1) {
      hipLaunchKernelGGL(cell_block_sum_kernel, dim3(nb), dim3(kCellThreads), 0, st, (const int*)count, ncell, bsum);
      if ((rc = check_launch())) return rc;
      hipLaunchKernelGGL(cell_block_scan_kernel, dim3(1), dim3(kBlockScanThreads), 0, st, bsum, nb, off + ncell);
      if ((rc = check_launch())) return rc;
    }
    hipLaunchKernelGGL(cell_scan_kernel, dim3(nb), dim3(kCellThreads), 0, st, (const int*)count, ncell,
                       nb > 1 ? (const int*)bsum : nullptr, off, nullptr, nb > 1 ? nullptr : off + ncell);
    if ((rc = check_launch())) return rc;
    if (n > 0) {
      hipLaunchKernelGGL(bin_points_kernel, dim3(grid_blocks(n, 256, device_cus() * 8)), dim3(256), 0, st,
                         (const int*)cell, (const int*)rank, (const int*)off, n, order);
      if ((rc = check_launch())) return rc;
    }
    const int sl = TC::slice(H), ng = n_groups(n);
    float* partial = (float*)ws + (size_t)nw * sl;
    hipLaunchKernelGGL(slice_sum_kernel, dim3((sl + 255) / 256, ng), dim3(256), 0, st, (const float*)ws, nw, sl,
                       partial);
    rc = check_launch();
    if (rc) return rc;
    // the latent gradient; the two-pass form writes its cell-corner sums over
    // the wave slices, which slice_sum_kernel has finished reading
    const long long nv = (long long)nd.R * nd.R * nd.R;
    // point subsets per cell: about one per 16 points of an average cell, at most 8
    int sub_log2 = 0;
    while (sub_log2 < 3 && (16LL << sub_log2) * ncell < n) ++sub_log2;
    if (nd.K == 1 && ((long long)ncell * 8 * F << sub_log2) <= (long long)nw * sl) {
      hipLaunchKernelGGL((cell_partials_kernel<F>),
                         dim3(grid_blocks(((long long)ncell << sub_log2) * (F / 4), 256, device_cus() * 32)), dim3(256),
                         0, st, xyz, nd.R, (long long)ncell, sub_log2, (const int*)off, (const int*)order,
                         (const float*)dz, (float*)ws);
      if ((rc = check_launch())) return rc;
      hipLaunchKernelGGL((vertex_sum_kernel<F>), dim3(grid_blocks(nv * (F / 4), 256, device_cus() * 32)), dim3(256), 0,
                         st, nd.R, sub_log2, (const float*)ws, d_latent);
      if ((rc = check_launch())) return rc;
    } else {
      // lanes per cell: about one per four points of an average cell, at most 8
      int lpc_log2 = 0;
      while (lpc_log2 < 3 && (4LL << lpc_log2) * ncell < n) ++lpc_log2;
      const long long nthreads = (long long)nd.K * nv * (8 << lpc_log2);
      hipLaunchKernelGGL((latent_grad_kernel<F>), dim3(grid_blocks(nthreads, 256, device_cus() * 32)), dim3(256), 0,
                         st, xyz, times, kt, nd.K, nd.R, nd.key_stride, (const int*)off, (const int*)order,
                         (const float*)dz, d_latent, lpc_log2);
      if ((rc = check_launch())) return rc;
    }
    const long long nwts = (long long)C * TC::G::K0IN + C + (long long)(H - 1) * (C * C + C) +
                           (long long)nd.NO * (C + 1);
    const float loss_scale = target && n > 0 ? 1.0f / (float)n : 1.0f;
    hipLaunchKernelGGL((gather_kernel<C, F, L, ACT, TE, FM>), dim3(grid_blocks(nwts + 1, 128, 1024)), dim3(128), 0, st, H,
                       nd.NO, (const float*)partial, ng, d_weights, out_loss, loss_scale);
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL((gather_long_kernel<C, F, L, ACT, TE, FM>), dim3((H - 1) * C + nd.NO + 1), dim3(64), 0, st, H,
                       nd.NO, (const float*)partial, ng, d_weights, out_loss, loss_scale);
    return check_launch();
  }
};

#define FV_TRAIN_CASES(X) \
  X(32, 8, 4)             \
  X(32, 16, 8)            \
  X(48, 8, 4)             \
  X(48, 16, 8)

// further (F, L) pairs: sine activation, no time encoding or Fourier matrix
#define FV_TRAIN_CASES_EXT(X) \
  X(32, 16, 4)                \
  X(32, 8, 8)                 \
  X(48, 16, 4)                \
  X(48, 8, 8)

// Training workspace for callers that cannot allocate device memory: one
// array per GPU, allocated with the code object and held until the process
// ends. Host code must not pass `scratch` itself to a kernel (on the host the
// name is only a stand-in for the device symbol); it uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticTrainScratchBytes];

}  // namespace

int static_train_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 2;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return 2;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return 0;
}

size_t train_workspace_bytes(const NetDev& nd, long long n) {
#define X(C_, F_, L_)                                                            \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_) {                                  \
    if (nd.time_enc == 1) return TrainEntry<C_, F_, L_, kSine, 1>::ws_bytes(nd, n); \
    if (nd.time_enc == 2) return TrainEntry<C_, F_, L_, kSine, 2>::ws_bytes(nd, n); \
    if (nd.time_enc == 3) return TrainEntry<C_, F_, L_, kSine, 3>::ws_bytes(nd, n); \
    if (nd.act == kSine) return TrainEntry<C_, F_, L_, kSine>::ws_bytes(nd, n);  \
    if (nd.act == kSnakeAlt) return TrainEntry<C_, F_, L_, kSnakeAlt>::ws_bytes(nd, n); \
    return TrainEntry<C_, F_, L_, kIdentity>::ws_bytes(nd, n);                   \
  }
  FV_TRAIN_CASES(X)
#undef X
#define X(C_, F_, L_)                                                                    \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_) {                                          \
    if (nd.act == kSine && nd.time_enc == 0 && !nd.fmat) return TrainEntry<C_, F_, L_, kSine>::ws_bytes(nd, n); \
    return 0;                                                                            \
  }
  FV_TRAIN_CASES_EXT(X)
#undef X
  return 0;
}

int launch_train(const NetDev& nd, const KeyTimes& kt, float* latent, float* weights, float* d_latent,
                 float* d_weights, const float* xyz, const float* times, long long n, const float* target,
                 const float* target_grad, float grad_weight, const float* dloss_dy, int use_adam, float lr_grid, float lr_mlp, float beta1, float beta2,
                 float eps, int step, float* m_lat, float* v_lat, float* m_w, float* v_w, float* out_loss,
                 void* workspace, size_t ws_bytes, int half, void* stream) {
  const hipStream_t st = (hipStream_t)stream;
  NetDev net = nd;
  net.weights = weights;
  int rc = 1;
#define FV_TRAIN_RUN(C_, F_, L_, ACT_, TE_, FM_)                                                             \
  rc = TrainEntry<C_, F_, L_, ACT_, TE_, FM_>::run(net, kt, latent, d_latent, d_weights, xyz, times, n, target,     \
                                              target_grad, grad_weight, dloss_dy, out_loss, workspace, half != 0, st)
#define X(C_, F_, L_)                                                        \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_) {                              \
    if (nd.time_enc != 0 || nd.fmat) {                                       \
      /* time encodings and Fourier matrices: sine activation, one at a time */ \
      if (nd.act != kSine || (nd.time_enc != 0 && nd.fmat)) rc = 1;          \
      else if (nd.fmat) FV_TRAIN_RUN(C_, F_, L_, kSine, 0, 1);               \
      else if (nd.time_enc == 1) FV_TRAIN_RUN(C_, F_, L_, kSine, 1, 0);      \
      else if (nd.time_enc == 2) FV_TRAIN_RUN(C_, F_, L_, kSine, 2, 0);      \
      else FV_TRAIN_RUN(C_, F_, L_, kSine, 3, 0);                            \
    } else if (nd.act == kSine) {                                            \
      FV_TRAIN_RUN(C_, F_, L_, kSine, 0, 0);                                 \
    } else if (nd.act == kSnakeAlt) {                                        \
      FV_TRAIN_RUN(C_, F_, L_, kSnakeAlt, 0, 0);                             \
    } else {                                                                 \
      FV_TRAIN_RUN(C_, F_, L_, kIdentity, 0, 0);                             \
    }                                                                        \
  }
  FV_TRAIN_CASES(X)
#undef X
#define X(C_, F_, L_)                                                                \
  if (nd.C == C_ && nd.F == F_ && nd.L == L_) {                                      \
    if (nd.act == kSine && nd.time_enc == 0 && !nd.fmat) FV_TRAIN_RUN(C_, F_, L_, kSine, 0, 0); \
    else rc = 1;                                                                     \
  }
  FV_TRAIN_CASES_EXT(X)
#undef X
#undef FV_TRAIN_RUN
  (void)ws_bytes;
  if (rc != 0 || !use_adam) return rc;
  const double bc1 = 1.0 - pow((double)beta1, (double)step);
  const double bc2 = 1.0 - pow((double)beta2, (double)step);
  const long long nlat = (long long)nd.K * nd.R * nd.R * nd.R * nd.F;
  static const int kTimeInputs[4] = {0, 1, 8, 9};
  const long long nw = (long long)nd.C * (3 + nd.F + 6 * nd.L + kTimeInputs[nd.time_enc]) + nd.C +
                       (long long)(nd.H - 1) * (nd.C * nd.C + nd.C) + (long long)nd.NO * (nd.C + 1);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_blocks(nlat, 256, device_cus() * 8)), dim3(256), 0, st, latent, d_latent,
                     m_lat, v_lat, nlat, (float)(lr_grid / bc1), beta1, beta2, (float)(1.0 / sqrt(bc2)), eps);
  rc = check_launch();
  if (rc) return rc;
  hipLaunchKernelGGL(adam_kernel, dim3(grid_blocks(nw, 256, device_cus() * 8)), dim3(256), 0, st, weights, d_weights,
                     m_w, v_w, nw, (float)(lr_mlp / bc1), beta1, beta2, (float)(1.0 / sqrt(bc2)), eps);
  return check_launch();
}

}  // namespace fvsrn_detail
