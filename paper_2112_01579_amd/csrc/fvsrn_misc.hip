// Dense-grid DVR (the uncompressed reference renderer), dense point sampling,
// Philox point sampling, grid casts, and the precision dispatch of the
// network launchers.
#include <stdio.h>

#include <atomic>
#include <mutex>

#include "fvsrn_common.hpp"

namespace fvsrn_detail {

namespace {

__device__ inline void tf_eval_d(const TFDev& tf, float d, float rgba[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) rgba[q] = tf.base[q];
  for (int j = 0; j < tf.n_seg; ++j) {
    const float w = __builtin_amdgcn_fmed3f(fmaf(d, tf.inv[j], tf.off[j]), 0.0f, 1.0f);
#pragma unroll
    for (int q = 0; q < 4; ++q) rgba[q] = fmaf(w, tf.delta[j][q], rgba[q]);
  }
}

__device__ inline int xcd_block_d(int nblocks) {
  const int b = blockIdx.x;
  if (nblocks % 8 != 0) return b;
  const int per = nblocks / 8;
  return (b % 8) * per + b / 8;
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
  const int tile = xcd_block_d(gridDim.x) * (kDenseThreads / 64) + wave;
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
    const float a0 = ray.t0 + (float)i * ray.ds;
    float a1 = ray.t0 + (float)(i + 1) * ray.ds;
    if (!fixed) a1 = fminf(a1, ray.t1);
    const float len = a1 - a0, tm = 0.5f * (a0 + a1);
    if (len <= 0.0f) break;
    const float sx = ray.o[0] + tm * ray.d[0];
    const float sy = ray.o[1] + tm * ray.d[1];
    const float sz = ray.o[2] + tm * ray.d[2];
    const float d = dense_sample(vol, nx, ny, nz, sx, sy, sz);
    float rgba[4];
    tf_eval_d(tf, d, rgba);
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
    unsigned long long mine = (unsigned long long)i, hit = (ray.hit && ray.nseg > 0) ? 1ull : 0ull;
    atomicAdd(stats, mine);
    atomicAdd(stats + 2, mine);
    if (hit) atomicAdd(stats + 1, 1ull);
  }
}

// Samples (out, nullable) and one-voxel central-difference gradients (out_g,
// nullable) of the dense grid, as the dense renderer shades.
__global__ void dense_points_kernel(const float* vol, int nx, int ny, int nz, const float* xyz,
                                    long long n, float* out, float* out_g) {
  const float hx = 2.0f / (float)(nx - 1), hy = 2.0f / (float)(ny - 1), hz = 2.0f / (float)(nz - 1);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    if (out) out[i] = dense_sample(vol, nx, ny, nz, x, y, z);
    if (out_g) {
      out_g[3 * i] = (dense_sample(vol, nx, ny, nz, x + hx, y, z) - dense_sample(vol, nx, ny, nz, x - hx, y, z)) /
                     (2.0f * hx);
      out_g[3 * i + 1] =
          (dense_sample(vol, nx, ny, nz, x, y + hy, z) - dense_sample(vol, nx, ny, nz, x, y - hy, z)) / (2.0f * hy);
      out_g[3 * i + 2] =
          (dense_sample(vol, nx, ny, nz, x, y, z + hz) - dense_sample(vol, nx, ny, nz, x, y, z - hz)) / (2.0f * hz);
    }
  }
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

}  // namespace

// Philox4x32-10 (Salmon et al., SC'11) of counter (i mod 2^32, i div 2^32,
// c_lo, c_hi) and key (k0, k1): four 32-bit outputs in c.
__device__ void philox4x32_10(long long i, uint32_t c_lo, uint32_t c_hi, uint32_t k0, uint32_t k1, uint32_t c[4]) {
  c[0] = (uint32_t)i;
  c[1] = (uint32_t)((unsigned long long)i >> 32);
  c[2] = c_lo;
  c[3] = c_hi;
  uint32_t k[2] = {k0, k1};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
}

namespace {

__global__ void sample_points_kernel(uint32_t k0, uint32_t k1, uint32_t c_lo, uint32_t c_hi,
                                     long long n, float* xyz) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    uint32_t c[4];
    philox4x32_10(i, c_lo, c_hi, k0, k1, c);
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

// SSIM map (Wang et al. 2004), one thread per output pixel; the 11 x 11
// Gaussian window is the outer product of the normalised 1-D weights.
struct Window11 {
  float g[11];
};

__global__ void ssim_kernel(const float4* a, const float4* b, int W, int H, int n, Window11 win, float* out) {
  const int WO = W - 10, HO = H - 10;
  const long long total = (long long)n * HO * WO;
  for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(o % WO), y = (int)((o / WO) % HO), img = (int)(o / ((long long)WO * HO));
    float m[3][5] = {};
    for (int i = 0; i < 11; ++i)
      for (int j = 0; j < 11; ++j) {
        const float w = win.g[i] * win.g[j];
        const long long p = ((long long)img * H + (y + i)) * W + (x + j);
        const float4 va = a[p], vb = b[p];
        const float pa[3] = {va.x, va.y, va.z}, pb[3] = {vb.x, vb.y, vb.z};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          m[ch][0] = fmaf(w, pa[ch], m[ch][0]);
          m[ch][1] = fmaf(w, pb[ch], m[ch][1]);
          m[ch][2] = fmaf(w, pa[ch] * pa[ch], m[ch][2]);
          m[ch][3] = fmaf(w, pb[ch] * pb[ch], m[ch][3]);
          m[ch][4] = fmaf(w, pa[ch] * pb[ch], m[ch][4]);
        }
      }
    const float C1 = 1e-4f, C2 = 9e-4f;
    float s = 0.0f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float mx = m[ch][0], my = m[ch][1];
      const float sx = m[ch][2] - mx * mx, sy = m[ch][3] - my * my, sxy = m[ch][4] - mx * my;
      s += ((2.0f * mx * my + C1) * (2.0f * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2));
    }
    out[o] = s * (1.0f / 3.0f);
  }
}

// uint8 quantisation (Sec. 4.2). One workgroup per channel finds the
// channel's minimum and maximum (order-independent, so exact) and writes
// (lo, (hi - lo) / 255); then every value is encoded as
// round-half-even((x - lo) / scale), clamped to [0, 255], in FP32.
__global__ __launch_bounds__(256) void channel_range_kernel(const float* src, long long n, int channels,
                                                            float* dequant) {
  __shared__ float s_lo[256], s_hi[256];
  const int ch = blockIdx.x, t = threadIdx.x;
  float lo = src[ch], hi = src[ch];
  for (long long i = t; i < n; i += blockDim.x) {
    const float x = src[i * channels + ch];
    lo = fminf(lo, x);
    hi = fmaxf(hi, x);
  }
  s_lo[t] = lo;
  s_hi[t] = hi;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      s_lo[t] = fminf(s_lo[t], s_lo[t + h]);
      s_hi[t] = fmaxf(s_hi[t], s_hi[t + h]);
    }
    __syncthreads();
  }
  if (t == 0) {
    dequant[2 * ch] = s_lo[0];
    dequant[2 * ch + 1] = (s_hi[0] - s_lo[0]) / 255.0f;
  }
}

__global__ void encode_u8_kernel(const float* src, long long count, int channels, const float* dequant,
                                 unsigned char* codes) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % channels);
    const float lo = dequant[2 * ch], scale = dequant[2 * ch + 1];
    float q = 0.0f;
    if (scale > 0.0f) q = fminf(fmaxf(rintf((src[i] - lo) / scale), 0.0f), 255.0f);
    codes[i] = (unsigned char)q;
  }
}

}  // namespace

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

namespace {
__device__ __align__(256) unsigned int tile_queues[2 * kTileQueueSlots];
}  // namespace

unsigned int* tile_queue_slot() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static unsigned int* base[kMaxDevices] = {};
  static std::atomic<unsigned int> next{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    snprintf(g_hip_err, sizeof(g_hip_err), "no current device for the tile queue");
    return nullptr;
  }
  unsigned int* b = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!base[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(tile_queues));
      if (e != hipSuccess || !p) {
        snprintf(g_hip_err, sizeof(g_hip_err), "tile queue: %s", hipGetErrorString(e));
        return nullptr;
      }
      base[dev] = static_cast<unsigned int*>(p);
    }
    b = base[dev];
  }
  return b + 2 * (next.fetch_add(1u) % kTileQueueSlots);
}

// ------------------------------------------ adaptive resampling (Sec. 5.4)

namespace {

// Position inside voxel v of a G^3 grid over [-1,1]^3 (x fastest) from three
// random words: p_a = fma((float)i_a + u_a, 2/G, -1), u_a = (r_a >> 8) 2^-24.
__device__ inline void voxel_position(int G, long long v, const uint32_t* r, float* p) {
  const long long iv[3] = {v % G, (v / G) % G, v / ((long long)G * G)};
  const float step = 2.0f / (float)G;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float u = (float)(r[a] >> 8) * 5.9604644775390625e-8f;  // 2^-24
    p[a] = fmaf((float)iv[a] + u, step, -1.0f);
  }
}

__global__ void voxel_points_kernel(uint32_t k0, uint32_t k1, uint32_t c_lo, uint32_t c_hi, int G, int per_voxel,
                                    long long n, float* xyz) {
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x) {
    uint32_t c[4];
    philox4x32_10(j, c_lo, c_hi, k0, k1, c);
    voxel_position(G, j / per_voxel, c, xyz + 3 * j);
  }
}

// E[v] = mean over the voxel's points of |network density - trilinear target|.
__global__ void error_reduce_kernel(const float* d, const float* vol, int nx, int ny, int nz, const float* xyz,
                                    long long n_voxels, int per_voxel, float* E) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n_voxels;
       v += (long long)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int k = 0; k < per_voxel; ++k) {
      const long long j = v * per_voxel + k;
      s += fabsf(d[j] - dense_sample(vol, nx, ny, nz, xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2]));
    }
    E[v] = s / (float)per_voxel;
  }
}

// Largest weight (bits of non-negative floats order like unsigned integers;
// entries that are not >= 0 count as 0). emax must start at 0.
__global__ void weight_max_kernel(const float* E, long long nv, unsigned* emax) {
  unsigned m = 0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
       v += (long long)gridDim.x * blockDim.x) {
    const float e = E[v];
    if (e >= 0.0f) m = max(m, __float_as_uint(e));
  }
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
  if ((threadIdx.x & 63) == 0 && m) atomicMax(emax, m);
}

constexpr int kScanThreads = 256, kScanItems = 8, kScanBlock = kScanThreads * kScanItems;

// Integer weights q_v = floor(E_v * (2^24 / max E)) and their inclusive
// prefix sums within each block of kScanBlock voxels; block totals to S.
__global__ __launch_bounds__(kScanThreads) void weight_scan_kernel(const float* E, long long nv, const unsigned* emax,
                                                                   unsigned long long* Q, unsigned long long* S) {
  __shared__ unsigned long long part[kScanThreads];
  const float em = __uint_as_float(*emax);
  const float scale = em > 0.0f ? 16777216.0f / em : 0.0f;
  const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
  unsigned long long q[kScanItems], run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const long long v = base + k;
    const float e = v < nv ? E[v] : 0.0f;
    run += (e >= 0.0f) ? (unsigned long long)floorf(e * scale) : 0ull;
    q[k] = run;
  }
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {  // inclusive scan of the thread totals
    const unsigned long long x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0ull;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  const unsigned long long before = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < nv) Q[base + k] = q[k] + before;
  if (threadIdx.x == kScanThreads - 1) S[blockIdx.x] = part[threadIdx.x];
}

// Exclusive prefix sums of the block totals (one workgroup, in place).
__global__ __launch_bounds__(kScanThreads) void block_offsets_kernel(unsigned long long* S, long long nb) {
  __shared__ unsigned long long part[kScanThreads];
  unsigned long long carry = 0;
  for (long long b0 = 0; b0 < nb; b0 += kScanThreads) {
    const long long b = b0 + threadIdx.x;
    const unsigned long long x = b < nb ? S[b] : 0ull;
    part[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const unsigned long long y = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0ull;
      __syncthreads();
      part[threadIdx.x] += y;
      __syncthreads();
    }
    if (b < nb) S[b] = carry + part[threadIdx.x] - x;
    const unsigned long long total = part[kScanThreads - 1];
    __syncthreads();
    carry += total;
  }
}

__global__ void add_offsets_kernel(unsigned long long* Q, long long nv, const unsigned long long* S) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
       v += (long long)gridDim.x * blockDim.x)
    Q[v] += S[v / kScanBlock];
}

// Point i (Philox counter words c_lo, c_hi): voxel v with
// Q[v-1] <= (r0 total) >> 32 < Q[v] (all weights zero: v = (r0 nv) >> 32),
// position inside it from r1..r3.
__device__ inline void draw_weighted(uint32_t k0, uint32_t k1, uint32_t c_lo, uint32_t c_hi,
                                     const unsigned long long* Q, unsigned long long total, int G, long long nv,
                                     long long i, float* out) {
  uint32_t c[4];
  philox4x32_10(i, c_lo, c_hi, k0, k1, c);
  long long v;
  if (total == 0) {
    v = (long long)(((unsigned long long)c[0] * (unsigned long long)nv) >> 32);
  } else {
    const unsigned long long target = __umul64hi((unsigned long long)c[0] << 32, total);
    long long lo = 0, hi = nv - 1;
    while (lo < hi) {
      const long long mid = (lo + hi) >> 1;
      if (Q[mid] > target) hi = mid;
      else lo = mid + 1;
    }
    v = lo;
  }
  voxel_position(G, v, c + 1, out);
}

__global__ void weighted_points_kernel(uint32_t k0, uint32_t k1, uint32_t c_lo, uint32_t c_hi,
                                       const unsigned long long* Q, int G, long long nv, long long n, float* xyz) {
  const unsigned long long total = Q[nv - 1];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    draw_weighted(k0, k1, c_lo, c_hi, Q, total, G, nv, i, xyz + 3 * i);
}

// Several grids' draws in one launch: point i of the batch belongs to grid
// k with start[k] <= i < start[k + 1], draws with counter + k and local
// index i - start[k] from the prefix sums at ws + k stride bytes.
struct MultiDraw {
  int n;
  long long start[kMaxDrawGrids + 1];
};

__global__ void weighted_points_multi_kernel(uint32_t k0, uint32_t k1, unsigned long long counter, const char* ws,
                                             unsigned long long stride, int G, long long nv, MultiDraw md,
                                             float* xyz) {
  const long long n = md.start[md.n];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    int k = 0;
#pragma unroll
    for (int j = 1; j < kMaxDrawGrids; ++j) k += (j < md.n && i >= md.start[j]) ? 1 : 0;
    const unsigned long long* Q = reinterpret_cast<const unsigned long long*>(ws + (unsigned long long)k * stride);
    const unsigned long long ck = counter + (unsigned long long)k;
    draw_weighted(k0, k1, (uint32_t)ck, (uint32_t)(ck >> 32), Q, Q[nv - 1], G, nv, i - md.start[k], xyz + 3 * i);
  }
}

__global__ void zero_u32_kernel(unsigned* p) { *p = 0u; }

}  // namespace

int launch_voxel_points(uint64_t seed, uint64_t counter, int G, int per_voxel, float* xyz, void* stream) {
  const long long n = (long long)G * G * G * per_voxel;
  hipLaunchKernelGGL(voxel_points_kernel, dim3(grid_blocks(n, 256, device_cus() * 16)), dim3(256), 0,
                     (hipStream_t)stream, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)counter,
                     (uint32_t)(counter >> 32), G, per_voxel, n, xyz);
  return check_launch();
}

int launch_error_reduce(const float* d, const float* vol, int nx, int ny, int nz, const float* xyz,
                        long long n_voxels, int per_voxel, float* E, void* stream) {
  hipLaunchKernelGGL(error_reduce_kernel, dim3(grid_blocks(n_voxels, 256, device_cus() * 16)), dim3(256), 0,
                     (hipStream_t)stream, d, vol, nx, ny, nz, xyz, n_voxels, per_voxel, E);
  return check_launch();
}

size_t weighted_points_workspace_bytes(long long nv) {
  const long long nb = (nv + kScanBlock - 1) / kScanBlock;
  return (size_t)(nv + nb) * 8 + 16;
}

int launch_weighted_points(uint64_t seed, uint64_t counter, const float* E, int G, long long n, float* xyz,
                           void* workspace, void* stream) {
  const hipStream_t st = (hipStream_t)stream;
  const long long nv = (long long)G * G * G, nb = (nv + kScanBlock - 1) / kScanBlock;
  unsigned long long* Q = (unsigned long long*)workspace;
  unsigned long long* S = Q + nv;
  unsigned* emax = (unsigned*)(S + nb);
  int rc = 0;
  if (E) {  // else the prefix sums of an earlier call are in the workspace
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, emax);
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(weight_max_kernel, dim3(grid_blocks(nv, 256, device_cus() * 8)), dim3(256), 0, st, E, nv,
                       emax);
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(weight_scan_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, E, nv, emax, Q, S);
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(block_offsets_kernel, dim3(1), dim3(kScanThreads), 0, st, S, nb);
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(add_offsets_kernel, dim3(grid_blocks(nv, 256, device_cus() * 8)), dim3(256), 0, st, Q, nv,
                       S);
    if ((rc = check_launch())) return rc;
  }
  if (n == 0) return 0;
  hipLaunchKernelGGL(weighted_points_kernel, dim3(grid_blocks(n, 256, device_cus() * 16)), dim3(256), 0, st,
                     (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)counter, (uint32_t)(counter >> 32), Q, G, nv,
                     n, xyz);
  return check_launch();
}

int launch_weighted_points_multi(uint64_t seed, uint64_t counter, int G, int n_grids, const int64_t* n_per_grid,
                                 float* xyz, const void* workspace, size_t stride, void* stream) {
  MultiDraw md;
  md.n = n_grids;
  md.start[0] = 0;
  for (int k = 0; k < n_grids; ++k) md.start[k + 1] = md.start[k] + n_per_grid[k];
  for (int k = n_grids + 1; k <= kMaxDrawGrids; ++k) md.start[k] = md.start[n_grids];
  const long long n = md.start[n_grids];
  if (n == 0) return 0;
  hipLaunchKernelGGL(weighted_points_multi_kernel, dim3(grid_blocks(n, 256, device_cus() * 16)), dim3(256), 0,
                     (hipStream_t)stream, (uint32_t)seed, (uint32_t)(seed >> 32), (unsigned long long)counter,
                     (const char*)workspace, (unsigned long long)stride, G, (long long)G * G * G, md, xyz);
  return check_launch();
}

const char* last_hip_error() { return g_hip_err; }

int launch_render(const NetDev& net, int prec, const TFDev& tf, const ViewBatch& views, const MarchDev& m,
                  float* out, unsigned long long* stats, void* stream) {
  switch (prec) {
    case kF32: return launch_render_p0(net, tf, views, m, out, stats, stream);
    case kF16: return launch_render_p1(net, tf, views, m, out, stats, stream);
    case kBF16: return launch_render_p2(net, tf, views, m, out, stats, stream);
  }
  return 1;
}

int launch_points(const NetDev& net, int prec, const float* xyz, long long n, int key, float key_w, float* out_d,
                  float* out_g, int gmode, void* stream) {
  switch (prec) {
    case kF32: return launch_points_p0(net, xyz, n, key, key_w, out_d, out_g, gmode, stream);
    case kF16: return launch_points_p1(net, xyz, n, key, key_w, out_d, out_g, gmode, stream);
    case kBF16: return launch_points_p2(net, xyz, n, key, key_w, out_d, out_g, gmode, stream);
  }
  return 1;
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
                        float* out_g, void* stream) {
  const int blocks = grid_blocks(n, 256, device_cus() * 16);
  hipLaunchKernelGGL(dense_points_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, vol, nx, ny, nz,
                     xyz, n, out, out_g);
  return check_launch();
}

int launch_sample_points(uint64_t seed, uint64_t counter, long long n, float* xyz, void* stream) {
  const int blocks = grid_blocks(n, 256, device_cus() * 16);
  hipLaunchKernelGGL(sample_points_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (uint32_t)seed,
                     (uint32_t)(seed >> 32), (uint32_t)counter, (uint32_t)(counter >> 32), n, xyz);
  return check_launch();
}

int launch_ssim(const float* a, const float* b, int width, int height, int n_images, float* out, void* stream) {
  Window11 win;
  double g[11], sum = 0.0;
  for (int i = 0; i < 11; ++i) {
    g[i] = exp(-(double)((i - 5) * (i - 5)) / (2.0 * 1.5 * 1.5));
    sum += g[i];
  }
  for (int i = 0; i < 11; ++i) win.g[i] = (float)(g[i] / sum);
  const long long total = (long long)n_images * (height - 10) * (width - 10);
  hipLaunchKernelGGL(ssim_kernel, dim3(grid_blocks(total, 256, device_cus() * 16)), dim3(256), 0,
                     (hipStream_t)stream, (const float4*)a, (const float4*)b, width, height, n_images, win, out);
  return check_launch();
}

int launch_quantize(const float* src, long long n, int channels, unsigned char* codes, float* dequant,
                    void* stream) {
  hipLaunchKernelGGL(channel_range_kernel, dim3(channels), dim3(256), 0, (hipStream_t)stream, src, n, channels,
                     dequant);
  int rc = check_launch();
  if (rc) return rc;
  const long long count = n * channels;
  hipLaunchKernelGGL(encode_u8_kernel, dim3(grid_blocks(count, 256, device_cus() * 16)), dim3(256), 0,
                     (hipStream_t)stream, src, count, channels, (const float*)dequant, codes);
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

}  // namespace fvsrn_detail
