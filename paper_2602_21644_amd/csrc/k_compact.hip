// gs_compact: order-preserving removal of the Gaussians a drop mask flags
// (the prune that follows the MP update of the mapping window), applied to
// any number of float planes of one length in one pass.
//
// Three launches over tiles of CP_TILE elements (each 256-thread workgroup
// takes a tile as CP_ROWS rows of 256 consecutive elements, so that every
// plane is read and written in coalesced rows):
//   count  : kept elements per tile (ballot + popcount per row);
//   scan   : one workgroup forms the exclusive tile offsets in a fixed order
//            and the total;
//   scatter: each tile ranks its elements (per-row ballot counts prefixed in
//            LDS, mbcnt inside the wave), copies every plane's kept elements
//            and places the scenes that begin in the tile.
// HBM bound: n (1 + 4 planes) bytes read, 4 planes bytes written per kept
// element.
#include "gs_internal.h"

namespace {

constexpr int CP_ROWS = 8;
constexpr int CP_TILE = GS_BLOCK * CP_ROWS;
constexpr int CP_WAVES = GS_BLOCK / 64;

struct PlaneTab {
  const float* src[GS_COMPACT_MAX_PLANES];
  float* dst[GS_COMPACT_MAX_PLANES];
  int32_t np;
};

struct SegTab {
  int64_t begin[GS_COMPACT_MAX_SEGS + 1];
  int32_t ns;  // segments; 0 = no segment output
};

__device__ __forceinline__ bool kept(const uint8_t* __restrict__ drop, int64_t i, int64_t n) {
  return i < n && drop[i] == 0;
}

__global__ __launch_bounds__(GS_BLOCK) void compact_count_kernel(const uint8_t* __restrict__ drop, int64_t n,
                                                                 uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_c[CP_WAVES];
  const int64_t base = (int64_t)blockIdx.x * CP_TILE;
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < CP_ROWS; ++r) {
    const uint64_t m = __ballot(kept(drop, base + r * GS_BLOCK + threadIdx.x, n));
    c += (uint32_t)__popcll(m);
  }
  if (__lane_id() == 0) s_c[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < CP_WAVES; ++w) t += s_c[w];
    cnt[blockIdx.x] = t;
  }
}

// One workgroup: off[b] = sum of cnt[0 .. b), in chunks of 1024 tiles with a
// running carry; then the total.
constexpr int CP_SCAN = 1024;
__global__ __launch_bounds__(CP_SCAN) void compact_scan_kernel(const uint32_t* __restrict__ cnt, int64_t ntile,
                                                               int64_t n, int64_t* __restrict__ off,
                                                               int64_t* __restrict__ n_out, SegTab seg,
                                                               int64_t* __restrict__ seg_out) {
  __shared__ int64_t s_w[CP_SCAN / 64];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int64_t b0 = 0; b0 < ntile; b0 += CP_SCAN) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t x = b < ntile ? (int64_t)cnt[b] : 0;
    // inclusive scan inside the wave
    int64_t y = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t t = __shfl_up(y, d, 64);
      if (lane >= d) y += t;
    }
    if (lane == 63) s_w[w] = y;
    __syncthreads();
    int64_t wo = 0;
    for (int i = 0; i < w; ++i) wo += s_w[i];
    const int64_t carry = s_carry;
    if (b < ntile) off[b] = carry + wo + y - x;
    __syncthreads();
    if (threadIdx.x == CP_SCAN - 1) s_carry = carry + wo + y;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *n_out = s_carry;
    // scenes that begin at n begin at the new total; the others are placed
    // by the scatter, which knows every element's rank
    for (int i = 0; i <= seg.ns && seg.ns > 0; ++i)
      if (seg.begin[i] >= n) seg_out[i] = s_carry;
  }
}

__global__ __launch_bounds__(GS_BLOCK) void compact_scatter_kernel(const uint8_t* __restrict__ drop, int64_t n,
                                                                   const int64_t* __restrict__ off, PlaneTab pt,
                                                                   SegTab seg, int64_t* __restrict__ seg_out) {
  __shared__ uint32_t s_c[CP_ROWS][CP_WAVES];
  const int64_t base = (int64_t)blockIdx.x * CP_TILE;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  bool k[CP_ROWS];
  uint32_t below[CP_ROWS];
#pragma unroll
  for (int r = 0; r < CP_ROWS; ++r) {
    k[r] = kept(drop, base + r * GS_BLOCK + threadIdx.x, n);
    const uint64_t m = __ballot(k[r]);
    below[r] = (uint32_t)__popcll(m & lanemask_lt());
    if (lane == 0) s_c[r][w] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  const int64_t o = off[blockIdx.x];
  int64_t d[CP_ROWS];
  uint32_t run = 0;
#pragma unroll
  for (int r = 0; r < CP_ROWS; ++r) {
    uint32_t before = run;
#pragma unroll
    for (int i = 0; i < CP_WAVES; ++i) {
      const uint32_t c = s_c[r][i];
      if (i < w) before += c;
      run += c;
    }
    d[r] = o + before + below[r];
  }
  // a scene that begins inside this tile begins at that element's rank (the
  // kept elements in front of it, whether or not it is kept itself)
  for (int i = 0; i <= seg.ns && seg.ns > 0; ++i) {
    const int64_t e = seg.begin[i] - base;
    if (e < 0 || e >= CP_TILE || seg.begin[i] >= n) continue;
    if ((int)(e % GS_BLOCK) != (int)threadIdx.x) continue;
    const int re = (int)(e / GS_BLOCK);
#pragma unroll
    for (int r = 0; r < CP_ROWS; ++r)
      if (r == re) seg_out[i] = d[r];
  }
  for (int p = 0; p < pt.np; ++p) {
    const float* __restrict__ src = pt.src[p];
    float* __restrict__ dst = pt.dst[p];
    float v[CP_ROWS];
#pragma unroll
    for (int r = 0; r < CP_ROWS; ++r) v[r] = k[r] ? src[base + r * GS_BLOCK + threadIdx.x] : 0.f;
#pragma unroll
    for (int r = 0; r < CP_ROWS; ++r)
      if (k[r]) dst[d[r]] = v[r];
  }
}

}  // namespace

size_t compact_ws_bytes(int64_t n) {
  const int64_t nt = (n + CP_TILE - 1) / CP_TILE;
  return (size_t)(nt * 4 + 255) / 256 * 256 + (size_t)nt * 8 + 8;
}

gs_status launch_compact(gs_ctx* ctx, const uint8_t* drop, int64_t n, int32_t n_planes, const float* const* src,
                         float* const* dst, const int64_t* seg_begin, int32_t n_seg, int64_t* seg_out,
                         int64_t* n_out, char* ws, hipStream_t s) {
  const int64_t nt = (n + CP_TILE - 1) / CP_TILE;
  uint32_t* cnt = (uint32_t*)ws;
  int64_t* off = (int64_t*)(ws + (size_t)(nt * 4 + 255) / 256 * 256);
  PlaneTab pt{};
  pt.np = n_planes;
  for (int p = 0; p < n_planes; ++p) {
    pt.src[p] = src[p];
    pt.dst[p] = dst[p];
  }
  SegTab sg{};
  sg.ns = seg_out ? n_seg : 0;
  for (int i = 0; seg_out && i <= n_seg; ++i) sg.begin[i] = seg_begin[i];
  if (nt > 0) GS_LAUNCH(ctx, compact_count_kernel, dim3((unsigned)nt), dim3(GS_BLOCK), 0, s, drop, n, cnt);
  GS_LAUNCH(ctx, compact_scan_kernel, dim3(1), dim3(CP_SCAN), 0, s, cnt, nt, n, off, n_out, sg, seg_out);
  if (nt > 0)
    GS_LAUNCH(ctx, compact_scatter_kernel, dim3((unsigned)nt), dim3(GS_BLOCK), 0, s, drop, n, off, pt, sg, seg_out);
  return gs_check_launch(ctx, "compact");
}
