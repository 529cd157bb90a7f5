// Device helpers shared by the two binning paths of gs_bin_sort.
#pragma once

#include "gs_internal.h"

// ------------------------------------------------------------------ exclusive scan (u32, in place)
static __device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_wave, uint32_t& total) {
  // inclusive wave scan with shuffles, then across the 4 waves through LDS
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (int i = 0; i < GS_BLOCK / 64; ++i) {
    const uint32_t t = s_wave[i];
    if (i < w) wbase += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return wbase + inc - x;
}

// ------------------------------------------------------------------ tile binning
// In-LDS 2D difference array of the tile rects of a set of records; after
// prefix sums over x then y each cell holds the number of rects covering it.
static __device__ __forceinline__ void diff_add(int* d, int stride, int x0, int y0, int x1, int y1) {
  atomicAdd(&d[y0 * stride + x0], 1);
  atomicAdd(&d[y0 * stride + x1 + 1], -1);
  atomicAdd(&d[(y1 + 1) * stride + x0], -1);
  atomicAdd(&d[(y1 + 1) * stride + x1 + 1], 1);
}

// Inclusive prefix of `len` ints at d[0], d[step], ... by one wave.
static __device__ __forceinline__ void wave_prefix(int* d, int step, int len) {
  const int lane = __lane_id();
  int carry = 0;
  for (int s = 0; s < len; s += 64) {
    const int i = s + lane;
    int x = i < len ? d[i * step] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    x += carry;
    if (i < len) d[i * step] = x;
    carry = __shfl(x, 63, 64);
  }
}

// Prefix over rows then columns of a (gy+1) x (gx+1) array, the work split
// over the waves [w0, w0 + nw) of the block.
static __device__ __forceinline__ void diff_integrate(int* d, int gx, int gy, int wave, int nwaves) {
  const int stride = gx + 1;
  for (int y = wave; y <= gy; y += nwaves) wave_prefix(d + y * stride, 1, gx + 1);
  __syncthreads();
  for (int x = wave; x <= gx; x += nwaves) wave_prefix(d + x, stride, gy + 1);
  __syncthreads();
}

static __device__ __forceinline__ void rect_of(int2 rc, int& x0, int& y0, int& x1, int& y1) {
  x0 = (int)(int16_t)(rc.x & 0xFFFF);
  y0 = (int)(int16_t)((uint32_t)rc.x >> 16);
  x1 = (int)(int16_t)(rc.y & 0xFFFF);
  y1 = (int)(int16_t)((uint32_t)rc.y >> 16);
}

// A caller's rect clipped to the view's gx x gy tile grid; false when empty
// after clipping. The full-list binning reads rects it did not write, and a
// rect outside the grid would index past its count arrays.
static __device__ __forceinline__ bool rect_clip(int2 rc, int gx, int gy, int& x0, int& y0, int& x1, int& y1) {
  rect_of(rc, x0, y0, x1, y1);
  x0 = max(x0, 0);
  y0 = max(y0, 0);
  x1 = min(x1, gx - 1);
  y1 = min(y1, gy - 1);
  return x0 <= x1 && y0 <= y1;
}

// Chunk processed by block b: spread consecutive chunks over the same XCD
// (blocks are dealt round-robin to the 8 XCDs) so that neighbouring count and
// list writes meet in one L2.
static __device__ __forceinline__ int chunk_of_block(int b, int nchunk) {
  const int per = (nchunk + 7) >> 3;
  const int c = (b & 7) * per + (b >> 3);
  return c;
}

