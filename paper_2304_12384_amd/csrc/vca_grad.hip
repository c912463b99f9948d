// vca_grad.hip -- differentiable luma texture energy E_Y and its temporal
// gradient h (Section 2 of the paper names both features) on gfx950.
//
// For gradients the transform's roundings are dropped: per w x w block X,
//   Y = C X C^T * 2^-(s1+s2),  s1 + s2 = 2 log2 w + B - 3,
//   H = sum W_ik |Y_ik| (DC and coefficients outside K x K weigh 0),
//   E = sum_blocks H / (C_Y w^2),  h_t = sum_blocks |H_t - H_{t-1}| / (C_Y w^2).
// d/dX of H is 2^-(s1+s2) C^T (W o sign(Y)) C, with sign(0) = 0.
//
// Layout (one wavefront per 32 x 32 tile, block-diagonal Cd for w < 32):
//   forward  T = X Cd^T, Y = Cd T: 16 + 2 x 16 v_mfma_f32_32x32x2f32, the
//            first accumulator feeding the second pass (split in hi and lo
//            parts) as its B operand;
//   backward S' = c o W o sign(Y) per block (c from dL/dE, dL/dh and the
//            signs of the neighbouring frames' block-energy differences),
//            V = Cd^T S' (chained), V through a per-wavefront LDS tile into
//            the A layout, G = V Cd, stored to dL/dX.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/vca.h"
#include "vca_host.h"
#include "vca_tile.h"

using namespace vca;

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

constexpr int kGWaves = 4;
constexpr int kGThreads = 64 * kGWaves;

// Per-lane FP32 operand tables (16 values per lane) and FP64 weights.
struct alignas(16) GradTables {
  float b1[64][16];   // stage 1 B: lane (k + 32g): Cd[k][16g + t]
  float a2[64][16];   // stage 2 A: lane (i + 32g): Cd[i][m_t(g)]
  float v1[64][16];   // backward V = Cd^T S: lane (m + 32g): Cd[m_t(g)][m]
  float g2[64][16];   // backward G = V Cd:  lane (n + 32g): Cd[16g + t][n]
  float wf[16][64];   // weight (FP32) of coefficient register j of each lane
  double wd[16][64];  // weight * 2^-(s1+s2) (FP64) for the energy sums
};

struct GradParams {
  const float* x;
  float* gx;
  double* blk_h;        // [frames][C_Y]
  const float* gE;      // [frames]
  const float* gh;      // [frames]
  const GradTables* tab;
  int64_t pitch;        // floats
  int64_t fstride;      // floats
  int32_t nbx, nby, ntx, tiles_per_frame, per_frame;
  FastDiv div_tpf, div_ntx;
  int32_t n_frames, seq_len;
  float grad_scale;     // 2^-(s1+s2) / (C_Y w^2)
};

template <int kW>
struct FTile {
  const float* base;    // tile origin in x
  int64_t origin;       // float offset of the tile origin (for gx)
  int32_t f, vr, vc, out0;
};

template <int kW>
__device__ inline FTile<kW> decode_ftile(const GradParams& p, int id) {
  constexpr int kBpt = kTile / kW;
  FTile<kW> t;
  t.f = (int)fastdiv((uint32_t)id, p.div_tpf);
  const int r = id - t.f * p.tiles_per_frame;
  const int ty = (int)fastdiv((uint32_t)r, p.div_ntx);
  const int tx = r - ty * p.ntx;
  const int by0 = ty * kBpt, bx0 = tx * kBpt;
  t.origin = t.f * p.fstride + (int64_t)by0 * kW * p.pitch + bx0 * kW;
  t.base = p.x + t.origin;
  t.vr = min(kBpt, p.nby - by0);
  t.vc = min(kBpt, p.nbx - bx0);
  t.out0 = t.f * p.per_frame + by0 * p.nbx + bx0;
  return t;
}

// Lane (r + 32 g) loads row r, samples 16g..16g+15 of the tile; rows and
// 16-byte pieces outside the valid blocks are redirected in bounds (a piece
// that starts inside the block grid lies inside the row's pitch).
template <int kW>
__device__ inline void load_ftile(const GradParams& p, const FTile<kW>& t, int lane, float x[16]) {
  const int r = lane & 31, g = lane >> 5;
  const int rows = t.vr * kW, cols = t.vc * kW;
  const float* row = t.base + (int64_t)(r < rows ? r : 0) * p.pitch;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int c = 16 * g + 4 * q;
    const v4f v = *reinterpret_cast<const v4f*>(row + (c < cols ? c : 0));
    x[4 * q + 0] = v[0];
    x[4 * q + 1] = v[1];
    x[4 * q + 2] = v[2];
    x[4 * q + 3] = v[3];
  }
}

// Y of a tile in the accumulator layout (lane = column, register j = row m_j),
// without the 2^-(s1+s2) scale.  For integer samples below 2^12 the first
// pass is exact in FP32; the second splits T = 4096 hi + lo (|lo| <= 2048,
// both exact) so that C hi and C lo are exact sums, and only their final
// combination rounds: sign(Y), and Y = 0, are exact.
__device__ inline v16f tile_y(const float b1[16], const float a2[16], const float x[16]) {
  v16f d = {};
#pragma unroll
  for (int t = 0; t < 16; t++) d = __builtin_amdgcn_mfma_f32_32x32x2f32(x[t], b1[t], d, 0, 0, 0);
  v16f yh = {}, yl = {};
#pragma unroll
  for (int t = 0; t < 16; t++) {
    const float hi = rintf(d[t] * (1.f / 4096.f));
    const float lo = fmaf(-4096.f, hi, d[t]);
    yh = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[t], hi, yh, 0, 0, 0);
    yl = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[t], lo, yl, 0, 0, 0);
  }
  v16f y;
#pragma unroll
  for (int j = 0; j < 16; j++) y[j] = fmaf(4096.f, yh[j], yl[j]);
  return y;
}

__device__ inline void load_row16(const float (*tab)[16], int lane, float out[16]) {
#pragma unroll
  for (int q = 0; q < 16; q += 4) {
    const v4f v = *reinterpret_cast<const v4f*>(&tab[lane][q]);
    out[q] = v[0];
    out[q + 1] = v[1];
    out[q + 2] = v[2];
    out[q + 3] = v[3];
  }
}

template <int kW, int kK>
__global__ __launch_bounds__(kGThreads) void energy_fwd_kernel(GradParams p) {
  constexpr int kBpt = kTile / kW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 31, g = lane >> 5;
  double wd[16];
#pragma unroll
  for (int j = 0; j < 16; j++) wd[j] = reg_used(j, kW, kK) ? p.tab->wd[j][lane] : 0.0;
  float b1[16], a2[16];
  load_row16(p.tab->b1, lane, b1);
  load_row16(p.tab->a2, lane, a2);
  const int total = p.n_frames * p.tiles_per_frame;
  for (int id = blockIdx.x * kGWaves + wave; id < total; id += gridDim.x * kGWaves) {
    const FTile<kW> t = decode_ftile<kW>(p, id);
    float x[16];
    load_ftile<kW>(p, t, lane, x);
    const v16f y = tile_y(b1, a2, x);
    double h[kBpt];
#pragma unroll
    for (int b = 0; b < kBpt; b++) h[b] = 0.0;
#pragma unroll
    for (int j = 0; j < 16; j++)
      if (reg_used(j, kW, kK)) h[(8 * (j / 4)) / kW] = fma(wd[j], (double)fabsf(y[j]), h[(8 * (j / 4)) / kW]);
#pragma unroll
    for (int off = 1; off < kW; off <<= 1)
#pragma unroll
      for (int b = 0; b < kBpt; b++) h[b] += __shfl_xor(h[b], off);
#pragma unroll
    for (int b = 0; b < kBpt; b++) h[b] += __shfl_xor(h[b], 32);
    if (g == 0 && r % kW == 0 && r / kW < t.vc) {
#pragma unroll
      for (int b = 0; b < kBpt; b++)
        if (b < t.vr) p.blk_h[t.out0 + b * p.nbx + r / kW] = h[b];
    }
  }
}

// One workgroup per frame: E and h from the block energies (fixed order).
__global__ __launch_bounds__(256) void energy_reduce_kernel(const double* blk_h, int32_t per_frame,
                                                            int32_t seq_len, double norm, float* E,
                                                            float* h) {
  __shared__ double red[2][256];
  const int f = blockIdx.x, t = threadIdx.x;
  const double* H = blk_h + (int64_t)f * per_frame;
  const bool first = f % seq_len == 0;
  double se = 0.0, sh = 0.0;
  for (int b = t; b < per_frame; b += 256) {
    se += H[b];
    if (!first) sh += fabs(H[b] - H[b - per_frame]);
  }
  red[0][t] = se;
  red[1][t] = sh;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    E[f] = (float)(red[0][0] * norm);
    h[f] = (float)(red[1][0] * norm);
  }
}

__device__ inline float sgn(double v) { return v > 0.0 ? 1.f : (v < 0.0 ? -1.f : 0.f); }

template <int kW, int kK>
__global__ __launch_bounds__(kGThreads) void energy_bwd_kernel(GradParams p) {
  constexpr int kBpt = kTile / kW;
  __shared__ float vt[kGWaves][32][33];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 31, g = lane >> 5;
  float wf[16];
#pragma unroll
  for (int j = 0; j < 16; j++) wf[j] = reg_used(j, kW, kK) ? p.tab->wf[j][lane] : 0.f;
  float b1[16], a2[16], v1[16], g2[16];
  load_row16(p.tab->b1, lane, b1);
  load_row16(p.tab->a2, lane, a2);
  load_row16(p.tab->v1, lane, v1);
  load_row16(p.tab->g2, lane, g2);
  const int total = p.n_frames * p.tiles_per_frame;
  for (int id = blockIdx.x * kGWaves + wave; id < total; id += gridDim.x * kGWaves) {
    const FTile<kW> t = decode_ftile<kW>(p, id);
    float x[16];
    load_ftile<kW>(p, t, lane, x);
    const v16f y = tile_y(b1, a2, x);
    // upstream coefficient of each block of this lane's block column
    const int f = t.f;
    const int pos = f % p.seq_len;
    const bool has_prev = pos > 0, has_next = pos + 1 < p.seq_len;
    const float gE = p.gE[f];
    const float ghf = has_prev ? p.gh[f] : 0.f;
    const float ghn = has_next ? p.gh[f + 1] : 0.f;
    const int bc = min(r / kW, t.vc - 1);
    float cb[kBpt];
#pragma unroll
    for (int b = 0; b < kBpt; b++) {
      const int idx = t.out0 + min(b, t.vr - 1) * p.nbx + bc;
      const double hc = p.blk_h[idx];
      float c = gE;
      if (has_prev) c += ghf * sgn(hc - p.blk_h[idx - p.per_frame]);
      if (has_next) c -= ghn * sgn(p.blk_h[idx + p.per_frame] - hc);
      cb[b] = c * p.grad_scale;
    }
    v16f s;
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const float sy = y[j] > 0.f ? 1.f : (y[j] < 0.f ? -1.f : 0.f);
      s[j] = cb[(8 * (j / 4)) / kW] * wf[j] * sy;
    }
    v16f v = {};
#pragma unroll
    for (int q = 0; q < 16; q++) v = __builtin_amdgcn_mfma_f32_32x32x2f32(v1[q], s[q], v, 0, 0, 0);
    // V[m_j][k] -> LDS row-major, then rows back in the A-operand layout
#pragma unroll
    for (int j = 0; j < 16; j++) vt[wave][reg_row(j, g)][r] = v[j];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float a[16];
#pragma unroll
    for (int q = 0; q < 16; q++) a[q] = vt[wave][r][16 * g + q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    v16f gm = {};
#pragma unroll
    for (int q = 0; q < 16; q++) gm = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], g2[q], gm, 0, 0, 0);
    // G[m_j][n]: lane n = r, row m_j; only pixels of valid blocks are written
    float* out = p.gx + t.origin;
    const int rows = t.vr * kW, cols = t.vc * kW;
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const int m = reg_row(j, g);
      if (m < rows && r < cols) out[(int64_t)m * p.pitch + r] = gm[j];
    }
  }
}

// Pixels outside the block grid (rows >= nby w, or columns >= nbx w) take no
// part in any block: their gradient is 0.  One grid-stride loop per frame.
__global__ __launch_bounds__(256) void zero_border_kernel(float* gx, int64_t pitch, int64_t fstride,
                                                          int32_t width, int32_t height,
                                                          int32_t grid_w, int32_t grid_h) {
  float* frame = gx + (int64_t)blockIdx.y * fstride;
  const int64_t bottom = (int64_t)(height - grid_h) * width;
  const int32_t right_w = width - grid_w;
  const int64_t total = bottom + (int64_t)grid_h * right_w;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    int64_t row, col;
    if (i < bottom) {
      row = grid_h + i / width;
      col = i % width;
    } else {
      const int64_t j = i - bottom;
      row = j / right_w;
      col = grid_w + j % right_w;
    }
    frame[row * pitch + col] = 0.f;
  }
}

void build_grad_tables(int w, int K, int bit_depth, GradTables& t) {
  std::vector<int8_t> b1, a2;
  std::vector<double> wt;
  build_tile_tables(w, K, b1, a2, wt);   // weights with DC and non-K x K at 0
  const double sc = std::ldexp(1.0, -(2 * ilog2c(w) + bit_depth - 3));
  for (int lane = 0; lane < 64; lane++) {
    const int c = lane & 31, g = lane >> 5;
    for (int q = 0; q < 16; q++) {
      const int mt = reg_row(q, g);
      t.b1[lane][q] = (float)matd(w, c, 16 * g + q);
      t.a2[lane][q] = (float)matd(w, c, mt);
      t.v1[lane][q] = (float)matd(w, mt, c);
      t.g2[lane][q] = (float)matd(w, 16 * g + q, c);
    }
    for (int j = 0; j < 16; j++) {
      t.wf[j][lane] = (float)wt[j * 64 + lane];
      t.wd[j][lane] = wt[j * 64 + lane] * sc;
    }
  }
}

using GradKernel = void (*)(GradParams);

template <int W>
GradKernel pick_grad(int K, bool bwd) {
  if (K == W) return bwd ? energy_bwd_kernel<W, W> : energy_fwd_kernel<W, W>;
  if (K == W / 2) return bwd ? energy_bwd_kernel<W, W / 2> : energy_fwd_kernel<W, W / 2>;
  if (K == W / 4) return bwd ? energy_bwd_kernel<W, W / 4> : energy_fwd_kernel<W, W / 4>;
  return nullptr;
}

GradKernel select_grad(int w, int K, bool bwd) {
  if (w == 32) return pick_grad<32>(K, bwd);
  if (w == 16) return pick_grad<16>(K, bwd);
  if (w == 8) return pick_grad<8>(K, bwd);
  return nullptr;
}

vca_status check_grad_config(const vca_grad_config* c) {
  if (!c || c->struct_size != sizeof(vca_grad_config)) return VCA_ERR_INVALID_ARG;
  const int w = c->block_size;
  if (w != 8 && w != 16 && w != 32) return VCA_ERR_INVALID_ARG;
  const int k = c->lowpass_k;
  if (k != 0 && k != w && k != w / 2 && k != w / 4) return VCA_ERR_INVALID_ARG;
  if (c->bit_depth != 8 && c->bit_depth != 10) return VCA_ERR_INVALID_ARG;
  if (c->width < w || c->height < w || c->n_seq <= 0 || c->seq_len <= 0 || c->device < 0)
    return VCA_ERR_INVALID_ARG;
  if ((int64_t)c->n_seq * c->seq_len > 65535) return VCA_ERR_INVALID_ARG;
  if (c->pitch < c->width || c->pitch % 4 || c->fstride % 4) return VCA_ERR_INVALID_ARG;
  if ((int64_t)c->n_seq * c->seq_len > 1 && c->fstride < c->pitch * c->height) return VCA_ERR_INVALID_ARG;
  const int64_t blocks = (int64_t)(c->width / w) * (c->height / w) * c->n_seq * c->seq_len;
  if (blocks > (int64_t)INT32_MAX / 2) return VCA_ERR_INVALID_ARG;
  return VCA_OK;
}

struct GradLaunch {
  GradParams p{};
  int n_frames = 0;
};

// Tables live in device memory per (w, K, bit depth); built once per process.
struct GradTableCache {
  std::mutex mu;
  std::map<std::tuple<int, int, int, int>, GradTables*> map;
};

GradTableCache& table_cache() {
  static GradTableCache c;
  return c;
}

vca_status get_tables(const vca_grad_config* c, int K, const GradTables** out) {
  GradTableCache& tc = table_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  const auto key = std::make_tuple(c->device, c->block_size, K, c->bit_depth);
  auto it = tc.map.find(key);
  if (it != tc.map.end()) {
    *out = it->second;
    return VCA_OK;
  }
  GradTables* h = new (std::nothrow) GradTables();
  if (!h) return VCA_ERR_OOM;
  build_grad_tables(c->block_size, K, c->bit_depth, *h);
  GradTables* d = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), sizeof(GradTables)) != hipSuccess) {
    delete h;
    return VCA_ERR_OOM;
  }
  const hipError_t e = hipMemcpy(d, h, sizeof(GradTables), hipMemcpyHostToDevice);
  delete h;
  if (e != hipSuccess) {
    (void)hipFree(d);
    return VCA_ERR_DEVICE;
  }
  tc.map[key] = d;   // kept until the process ends
  *out = d;
  return VCA_OK;
}

vca_status prepare(const vca_grad_config* c, const float* x, GradLaunch& L) {
  vca_status s = check_grad_config(c);
  if (s != VCA_OK) return s;
  if (!x || ((uintptr_t)x & 15)) return VCA_ERR_INVALID_ARG;
  const int w = c->block_size, K = c->lowpass_k == 0 ? w : c->lowpass_k;
  const int bpt = kTile / w;
  GradParams& p = L.p;
  p.x = x;
  p.pitch = c->pitch;
  p.fstride = c->fstride;
  p.nbx = c->width / w;
  p.nby = c->height / w;
  p.ntx = (p.nbx + bpt - 1) / bpt;
  p.tiles_per_frame = p.ntx * ((p.nby + bpt - 1) / bpt);
  p.per_frame = p.nbx * p.nby;
  p.div_tpf = make_fastdiv((uint32_t)p.tiles_per_frame);
  p.div_ntx = make_fastdiv((uint32_t)p.ntx);
  p.n_frames = c->n_seq * c->seq_len;
  p.seq_len = c->seq_len;
  p.grad_scale = (float)(std::ldexp(1.0, -(2 * ilog2c(w) + c->bit_depth - 3)) /
                         ((double)p.per_frame * w * w));
  L.n_frames = p.n_frames;
  return get_tables(c, K, &p.tab);
}

vca_status launch_grad(const vca_grad_config* c, const GradParams& p, bool bwd, hipStream_t st) {
  const int w = c->block_size, K = c->lowpass_k == 0 ? w : c->lowpass_k;
  GradKernel kern = select_grad(w, K, bwd);
  if (!kern) return VCA_ERR_UNSUPPORTED;
  int resident = 0, dev = 0;
  hipDeviceProp_t prop;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kern, kGThreads, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return VCA_ERR_DEVICE;
  const int64_t groups = ((int64_t)p.n_frames * p.tiles_per_frame + kGWaves - 1) / kGWaves;
  const int grid = (int)std::min<int64_t>(groups, (int64_t)prop.multiProcessorCount * std::max(1, resident));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kGThreads), 0, st, p);
  return hipGetLastError() == hipSuccess ? VCA_OK : VCA_ERR_DEVICE;
}

}  // namespace

extern "C" {

int64_t vca_grad_workspace(const vca_grad_config* c) {
  if (check_grad_config(c) != VCA_OK) return -1;
  return (int64_t)(c->width / c->block_size) * (c->height / c->block_size) * c->n_seq * c->seq_len;
}

vca_status vca_energy_forward(const vca_grad_config* c, const float* x, float* E, float* h,
                              double* workspace, void* hip_stream) {
  if (!x || ((uintptr_t)x & 15) || !E || !h || !workspace) return VCA_ERR_INVALID_ARG;
  GradLaunch L;
  vca_status s = check_grad_config(c);
  if (s != VCA_OK) return s;
  DeviceGuard guard(c->device);
  if ((s = prepare(c, x, L)) != VCA_OK) return s;
  L.p.blk_h = workspace;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if ((s = launch_grad(c, L.p, false, st)) != VCA_OK) return s;
  const double norm = 1.0 / ((double)L.p.per_frame * c->block_size * c->block_size);
  hipLaunchKernelGGL(energy_reduce_kernel, dim3(L.n_frames), dim3(256), 0, st, workspace,
                     L.p.per_frame, L.p.seq_len, norm, E, h);
  return hipGetLastError() == hipSuccess ? VCA_OK : VCA_ERR_DEVICE;
}

vca_status vca_energy_backward(const vca_grad_config* c, const float* x, const double* workspace,
                               const float* grad_E, const float* grad_h, float* grad_x,
                               void* hip_stream) {
  if (!x || ((uintptr_t)x & 15) || !workspace || !grad_E || !grad_h || !grad_x ||
      ((uintptr_t)grad_x & 15))
    return VCA_ERR_INVALID_ARG;
  GradLaunch L;
  vca_status s = check_grad_config(c);
  if (s != VCA_OK) return s;
  DeviceGuard guard(c->device);
  if ((s = prepare(c, x, L)) != VCA_OK) return s;
  L.p.blk_h = const_cast<double*>(workspace);
  L.p.gE = grad_E;
  L.p.gh = grad_h;
  L.p.gx = grad_x;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if ((s = launch_grad(c, L.p, true, st)) != VCA_OK) return s;
  const int w = c->block_size;
  const int grid_w = L.p.nbx * w, grid_h = L.p.nby * w;
  const int64_t border = (int64_t)(c->height - grid_h) * c->width + (int64_t)grid_h * (c->width - grid_w);
  if (border > 0) {
    const int gx_blocks = (int)std::min<int64_t>((border + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_border_kernel, dim3(gx_blocks, L.n_frames), dim3(256), 0, st, grad_x,
                       c->pitch, c->fstride, c->width, c->height, grid_w, grid_h);
    if (hipGetLastError() != hipSuccess) return VCA_ERR_DEVICE;
  }
  return VCA_OK;
}

}  // extern "C"
