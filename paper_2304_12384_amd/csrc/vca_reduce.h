// vca_reduce.h -- per-frame reduction of block energies and DC terms into
// the seven features of Section 2 of the paper (E_Y, h, L_Y, E_U, E_V, L_U,
// L_V), shared by the plain and the batched paths.
//
// One workgroup per frame: each thread sums a fixed strided subset of the
// frame's blocks in FP64, then a fixed LDS tree combines the threads, so the
// result is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vca {

constexpr int kReduceThreads = 1024;   // a power of two
static_assert((kReduceThreads & (kReduceThreads - 1)) == 0, "first_at uses a mask");

struct ReduceParams {
  const double* blk_h;     // block energies of frame 0 of the launch
  const int32_t* blk_dc;   // block DC terms, same layout
  const double* state_in;  // luma H of the frame before frame 0, or null (h = 0)
  double* state_out;       // receives luma H of the last frame
  float* ring;             // [capacity][7] feature ring
  int32_t* frame_err;      // per frame of the launch: validation mark of the forward
                           // kernel (moved to err_ring and cleared), or null
  int32_t* err_ring;       // [capacity] validation marks beside the feature ring
  int64_t first_frame;     // global index of frame 0 of this launch
  int64_t capacity;
  int32_t cnt[3];          // blocks per plane
  int32_t per_frame;
  int32_t n_frames;
  int32_t frame_begin;     // batched form: first reduce workgroup of this stream
  int32_t pad;
  double inv_norm[3];      // 1 / (C_P w^2)
};

__device__ inline void reduce_frame(const ReduceParams& p, int f) {
  __shared__ double red[7][kReduceThreads];
  const int t = threadIdx.x;
  const double* H = p.blk_h + (int64_t)f * p.per_frame;
  const int32_t* DC = p.blk_dc + (int64_t)f * p.per_frame;
  const double* prev = f > 0 ? H - p.per_frame : p.state_in;
  double s[7] = {0, 0, 0, 0, 0, 0, 0};   // H_Y H_U H_V L_Y L_U L_V dH
  const int e0 = p.cnt[0], e1 = p.cnt[0] + p.cnt[1];
  // The thread's blocks b = t, t + N, ... (N = kReduceThreads), plane by
  // plane: each sum sees its blocks in the same order as one loop over all
  // of them would, without selecting the plane per block.
  auto first_at = [&](int e) { return e + ((t - e) & (kReduceThreads - 1)); };
  for (int b = t; b < e0; b += kReduceThreads) {
    const double hb = H[b];
    s[0] += hb;
    s[3] += sqrt((double)DC[b]);
    if (prev) s[6] += fabs(hb - prev[b]);
  }
  for (int b = first_at(e0); b < e1; b += kReduceThreads) {
    s[1] += H[b];
    s[4] += sqrt((double)DC[b]);
  }
  for (int b = first_at(e1); b < p.per_frame; b += kReduceThreads) {
    s[2] += H[b];
    s[5] += sqrt((double)DC[b]);
  }
#pragma unroll
  for (int q = 0; q < 7; q++) red[q][t] = s[q];
  __syncthreads();
  for (int w = kReduceThreads / 2; w >= 1; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int q = 0; q < 7; q++) red[q][t] += red[q][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int64_t slot = (p.first_frame + f) % p.capacity;
    if (p.frame_err) {
      p.err_ring[slot] = p.frame_err[f];
      p.frame_err[f] = 0;   // clean for the next launch on this stream
    }
    float* o = p.ring + slot * 7;
    o[0] = (float)(red[0][0] * p.inv_norm[0]);
    o[1] = (float)(red[6][0] * p.inv_norm[0]);
    o[2] = (float)(red[3][0] * p.inv_norm[0]);
    o[3] = (float)(red[1][0] * p.inv_norm[1]);
    o[4] = (float)(red[2][0] * p.inv_norm[2]);
    o[5] = (float)(red[4][0] * p.inv_norm[1]);
    o[6] = (float)(red[5][0] * p.inv_norm[2]);
  }
  if (f == p.n_frames - 1)
    for (int b = t; b < p.cnt[0]; b += kReduceThreads) p.state_out[b] = H[b];
}

}  // namespace vca
