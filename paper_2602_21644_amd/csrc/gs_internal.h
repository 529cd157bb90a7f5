// Internal definitions shared by the gfx950 kernels and the host dispatch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/gs.h"

#define GS_BLOCK 256

// Per-batch view table, passed by value to every kernel (fits the kernel
// argument segment). Record offsets are multiples of 64 so a wave of records
// never straddles two views.
struct ViewTab {
  int32_t nv;
  int32_t ntiles;   // total tiles over views
  int64_t nrec;     // total records (padded)
  int64_t npix;     // total pixels
  int64_t ng;       // total Gaussians (all scenes)
  int32_t W[GS_MAX_VIEWS], H[GS_MAX_VIEWS], gx[GS_MAX_VIEWS], gy[GS_MAX_VIEWS];
  int32_t tile_base[GS_MAX_VIEWS + 1];
  int32_t scene[GS_MAX_VIEWS];
  int64_t n[GS_MAX_VIEWS];      // Gaussians of the view's scene
  int64_t npad[GS_MAX_VIEWS];   // n rounded up to 64
  int64_t g_off[GS_MAX_VIEWS];  // first Gaussian of the view's scene
  int64_t r_off[GS_MAX_VIEWS];  // first record of the view
  int64_t px_off[GS_MAX_VIEWS]; // first pixel of the view
};

// Binning layout (per view), also by value.
struct BinTab {
  int32_t chunk;                  // records per chunk (4 waves x chunk/4)
  int32_t nchunk[GS_MAX_VIEWS];   // chunks of the view (>= 1)
  int64_t nlim[GS_MAX_VIEWS];     // records binned: min(max_rank, npad)
  int64_t cm_off[GS_MAX_VIEWS];   // offset of the view in the count matrix
  int32_t sblk[GS_MAX_VIEWS];     // radix blocks of the view
  int64_t h_off[GS_MAX_VIEWS];    // offset of the view in the radix histogram
  int32_t truncated[GS_MAX_VIEWS];
};

__device__ __forceinline__ int view_of_tile(const ViewTab& tab, int t) {
  int v = 0;
  for (int i = 1; i < tab.nv; ++i)
    if (t >= tab.tile_base[i]) v = i;
  return v;
}

// The compositing record stores the conic in base-2 exponent units:
// (c1, c2, c3) = (-k1 log2(e) / 2, -k2 log2(e), -k3 log2(e) / 2), so that the
// Gaussian's value at offset (dx, dy) = u - pixel is exp2 of
//   c1 dx^2 + c2 dx dy + c3 dy^2 = dx (c1 dx + c2 dy) + c3 dy^2,
// evaluated with every rounding spelled out (explicit fma, no contractible
// mul+add), so the forward and the backward kernels compute bit-identical
// alphas and take identical skips.
#define GS_LOG2E 1.4426950408889634f
__device__ __forceinline__ float gs_conic_scale_diag(float k) { return -0.5f * GS_LOG2E * k; }
__device__ __forceinline__ float gs_conic_scale_off(float k) { return -GS_LOG2E * k; }
__device__ __forceinline__ float gs_power2(float c1, float c2, float c3, float dx, float dy) {
  const float t = __builtin_fmaf(c2, dy, c1 * dx);
  const float u = c3 * dy;
  return __builtin_fmaf(t, dx, u * dy);
}

#define GS_ALPHA_MIN (1.0f / 255.0f)
#define GS_ALPHA_MAX 0.99f
#define GS_T_MIN 1e-4f

// DPP wave64 reduction: returns the sum over all 64 lanes in lane 63.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf, bool BOUND = true>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, BANK_MASK, BOUND));
}

__device__ __forceinline__ float wave_sum_to_lane63(float x) {
  x += dpp_mov<0x111>(x);               // row_shr:1
  x += dpp_mov<0x112>(x);               // row_shr:2
  x += dpp_mov<0x114>(x);               // row_shr:4 -> lane i holds the sum of lanes i-7..i
  x += dpp_mov<0x118>(x);               // row_shr:8 -> lane 15 of each row holds the row sum
  x += dpp_mov<0x142, 0xa>(x);          // row_bcast:15 -> rows 1, 3 add the previous row's lane 15
  x += dpp_mov<0x143, 0xc>(x);          // row_bcast:31 -> rows 2, 3 add lane 31
  return x;
}

// Sums each of ten per-lane values over the 64 lanes of a wave (all lanes
// active). A transposed reduction: the two permlane swaps halve the values per
// lane twice while folding lanes 32 and 16 apart, then three in-row DPP
// chains finish. The totals land in lane 15 of every row r (lanes 15, 31, 47,
// 63) as k[0..2]:
//   row 0: (v0, v2, v4)   row 1: (v1, v3, 0)
//   row 2: (v5, v7, v9)   row 3: (v6, v8, 0)
__device__ __forceinline__ void wave_sum10(const float v[10], float k[3]) {
  float h[6];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    // lanes 0-31 end up with v[i] folded over lanes +32, lanes 32-63 with v[i+5]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 5]), false, false);
    h[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  h[5] = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // rows 0 and 2 take h[2i] folded over rows +1, rows 1 and 3 take h[2i+1]
    const auto r =
        __builtin_amdgcn_permlane16_swap(__float_as_uint(h[2 * i]), __float_as_uint(h[2 * i + 1]), false, false);
    k[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) k[i] += dpp_mov<0x111>(k[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) k[i] += dpp_mov<0x112>(k[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) k[i] += dpp_mov<0x114>(k[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) k[i] += dpp_mov<0x118>(k[i]);
}

// The same transposed reduction for six values (the terms a pose-only
// backward needs). Totals in lane 15 of every row r as k[0..1]:
//   row 0: (v0, v2)   row 1: (v1, 0)   row 2: (v3, v5)   row 3: (v4, 0)
__device__ __forceinline__ void wave_sum6(const float v[6], float k[2]) {
  float h[4];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // lanes 0-31 end up with v[i] folded over lanes +32, lanes 32-63 with v[i+3]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 3]), false, false);
    h[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  h[3] = 0.f;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    // rows 0 and 2 take h[2i] folded over rows +1, rows 1 and 3 take h[2i+1]
    const auto r =
        __builtin_amdgcn_permlane16_swap(__float_as_uint(h[2 * i]), __float_as_uint(h[2 * i + 1]), false, false);
    k[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) k[i] += dpp_mov<0x111>(k[i]);
#pragma unroll
  for (int i = 0; i < 2; ++i) k[i] += dpp_mov<0x112>(k[i]);
#pragma unroll
  for (int i = 0; i < 2; ++i) k[i] += dpp_mov<0x114>(k[i]);
#pragma unroll
  for (int i = 0; i < 2; ++i) k[i] += dpp_mov<0x118>(k[i]);
}

// Sum of x over the 64 lanes of a wave, returned in every lane (an xor
// butterfly of shuffles: a fixed order per lane, so repeat calls agree).
__device__ __forceinline__ double wave_sum_all_d(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Loss arguments of one call (Eq. 20-22 with the lambda1/lambda2 weights):
// targets, weights, adjoint outputs (dM, dT nullable) and the float64
// partials. Cg == nullptr means no loss.
struct LossArgs {
  const float *Cg, *Dg;
  float lp, ld, epsA;
  int wmode, gtw;
  float *dC, *dD, *dM, *dT;
  double* part;  // float64 partials
  float* loss;   // [views] totals
};

__device__ __forceinline__ float loss_sgn(float x) { return (float)((x > 0.f) - (x < 0.f)); }

// One pixel p (planar index, P pixels in all) with rendered colour c, depth D,
// MP m and transmittance T against target colour g and depth dg (0: none):
// writes its adjoints and returns its loss term w * (lp |c - g|_1 +
// ld [dg > 0] |D - dg|).
__device__ __forceinline__ double pixel_loss(const LossArgs& la, int64_t P, int64_t p, float c0, float c1, float c2,
                                             float D, float m, float T, float g0, float g1, float g2, float dg) {
  const float A = 1.0f - T;
  bool ok;
  float w;
  if (la.wmode == 0) {
    ok = A > la.epsA;
    w = ok ? 1.0f - m / A : 0.0f;
  } else {
    ok = true;
    w = A - m;
  }
  const float r0 = c0 - g0, r1 = c1 - g1, r2 = c2 - g2;
  const float rd = dg > 0.f ? D - dg : 0.f;
  // one explicit fma, so that every kernel using this rounds it alike
  const float per = fmaf(la.ld, fabsf(rd), la.lp * (fabsf(r0) + fabsf(r1) + fabsf(r2)));
  const float lw = la.lp * w;
  la.dC[p] = lw * loss_sgn(r0);
  la.dC[P + p] = lw * loss_sgn(r1);
  la.dC[2 * P + p] = lw * loss_sgn(r2);
  la.dD[p] = la.ld * w * loss_sgn(rd);
  if (la.dM || la.dT) {
    float gm = 0.f, gt = 0.f;
    if (la.gtw) {
      if (la.wmode == 0) {
        if (ok) {
          gm = -per / A;
          gt = -per * m / (A * A);
        }
      } else {
        gm = -per;
        gt = -per;
      }
    }
    if (la.dM) la.dM[p] = gm;
    if (la.dT) la.dT[p] = gt;
  }
  return (double)w * (double)per;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }

// Host helpers
struct GsTimer {
  const char* name;
  hipEvent_t a, b;
};

struct gs_ctx {
  int device;
  int render_batch;
  int bwd_batch;
  int bin_chunk;
  int timing;                    // 1: bracket every launch with HIP events
  int tile_order;                // 1: backward tiles heaviest first when tile_work is given
  int bwd_copies;                // accumulators of the backward's 2D adjoint (1, 2, 4, 8)
  int wave_cull;                 // 1: each wave skips the entries that cannot reach its 16x4 strip
  int n_cu;                      // compute units of the device (0: not queried yet)
  int proj_resident;             // bwd_project blocks the device holds at once (0: not queried yet)
  size_t lds_limit;              // LDS per workgroup usable by the binning scatter (0: not queried)
  int no_alloc;                  // 1 inside an allocation-free call: launches are not timed
  int exact_keys;                // 1: the prefix path's projection runs the exact test on every Gaussian
  std::vector<GsTimer> pending;  // launches whose events are not read yet
  char err[512];
};

// Kernel launch; with ctx->timing set, records a start and a stop event on the
// launch stream around it (measurement only: not for graph capture), under
// the kernel's name or the given one.
#define GS_LAUNCH(ctx, kern, grid, block, shm, strm, ...) \
  GS_LAUNCH_NAMED(ctx, #kern, kern, grid, block, shm, strm, __VA_ARGS__)
#define GS_LAUNCH_NAMED(ctx, name, kern, grid, block, shm, strm, ...)      \
  do {                                                                      \
    hipEvent_t e0_ = nullptr, e1_ = nullptr;                                \
    const bool t_ = (ctx) && (ctx)->timing && !(ctx)->no_alloc;             \
    if (t_) {                                                               \
      (void)hipEventCreate(&e0_);                                           \
      (void)hipEventCreate(&e1_);                                           \
      (void)hipEventRecord(e0_, strm);                                      \
    }                                                                       \
    hipLaunchKernelGGL(kern, grid, block, shm, strm, __VA_ARGS__);          \
    if (t_) {                                                               \
      (void)hipEventRecord(e1_, strm);                                      \
      gs_note_timer(ctx, name, e0_, e1_);                                   \
    }                                                                       \
  } while (0)

// Keeps a timed launch's events for gs_ctx_kernel_times (drops them if the
// record cannot grow: no exception leaves the library).
void gs_note_timer(gs_ctx* ctx, const char* name, hipEvent_t a, hipEvent_t b);

gs_status gs_fail(gs_ctx* ctx, gs_status s, const char* fmt, ...);
gs_status gs_check_launch(gs_ctx* ctx, const char* what);

// Workspace layout of gs_bin_sort (byte offsets, 256-aligned).
struct BinWs {
  size_t keys_a, keys_b, vals_a, vals_b, hist, part, total, cm, bytes;
  int64_t hist_n, cm_n;
};

// Launchers (one translation unit each).
gs_status launch_project(gs_ctx*, const ViewTab&, const gs_camera*, const gs_gaussians*, gs_proj*, hipStream_t);
void bin_tab_fill(const ViewTab&, int, int64_t, BinTab&);
BinWs bin_ws_layout(const ViewTab&, const BinTab&);
gs_status launch_bin_sort(gs_ctx*, const ViewTab&, const BinTab&, const gs_proj*, gs_bins*, char*, hipStream_t);
// with `loss` set, the loss of Eq. (20)-(22) is fused into the forward's
// epilogue: the pixel adjoints and one float64 partial per tile
gs_status launch_render_fwd(gs_ctx*, const ViewTab&, const gs_proj*, const gs_bins*, const float*, gs_image*,
                            hipStream_t, const LossArgs* loss = nullptr);
// The Gaussians the backward's tile pass gave a gradient: flag[N] (0 or 1,
// zero on entry, cleared again by the projection adjoint), the list of
// flagged Gaussians in the order they were flagged, its length, and the
// ticket that finds the projection adjoint's last working workgroup (both
// zero on entry and reset by that workgroup).
struct TouchArgs {
  uint32_t* flag;
  uint32_t* list;
  uint32_t* count;
  uint32_t* ticket;
};
gs_status launch_render_bwd_tiles(gs_ctx*, const ViewTab&, const gs_proj*, const gs_bins*, const gs_image*,
                                  const gs_pixel_grads*, const float*, float*, TouchArgs, const gs_grads*,
                                  hipStream_t);
gs_status launch_bwd_project(gs_ctx*, const ViewTab&, const gs_camera*, const gs_gaussians*, float*, TouchArgs,
                             float*, gs_grads*, hipStream_t);
constexpr int kChainBlocks = 256;  // workgroups of the projection adjoint that walk the list
int loss_blocks(const ViewTab&);
LossArgs loss_args(const gs_target*, const gs_loss_params*, gs_pixel_grads*, double* part, float* loss);
gs_status launch_loss(gs_ctx*, const ViewTab&, const gs_image*, const gs_target*, const gs_loss_params*, float*,
                      gs_pixel_grads*, double*, hipStream_t);
size_t bin_prefix_ws_bytes(gs_ctx*, const ViewTab&, int64_t capacity);
int64_t bin_prefix_cap();
gs_status launch_bin_prefix(gs_ctx*, const ViewTab&, const gs_camera*, const gs_gaussians*, const gs_proj*,
                            gs_bins*, char*, hipStream_t);
size_t mp_ws_bytes(const ViewTab&, int64_t npix);
gs_status launch_mp_update(gs_ctx*, const ViewTab&, const gs_proj*, const gs_image*, const gs_target*,
                           const gs_mp_frame*, const gs_mp_params*, float*, gs_mp_out*, char*, hipStream_t);
size_t mp_reg_ws_bytes(int64_t n);
gs_status launch_mp_reg(gs_ctx*, int64_t n, const float* mean, const float* prev, const float* mp, const float* T,
                        float lam, float* loss, float* dmean, double* part, hipStream_t);
size_t edge_warp_ws_bytes(const ViewTab&, int32_t n_pairs);
gs_status launch_epipolar(gs_ctx*, const gs_camera* cams, int v1, int v2, const float* p1, const float* p2,
                          int64_t m, const int32_t* ids, const int64_t* seg, int64_t K, int64_t n, float eps,
                          float tau, float mp_restore, float* d, float* dbar, uint8_t* state, float* mp,
                          hipStream_t s);
gs_status launch_edge_warp(gs_ctx*, const ViewTab&, const gs_camera*, const gs_image*, const gs_target*,
                           const gs_edge_pair*, int32_t, const gs_edge_params*, float* loss, float* ddepth,
                           float* dpose, double* part, hipStream_t);
size_t compact_ws_bytes(int64_t n);
gs_status launch_compact(gs_ctx*, const uint8_t* drop, int64_t n, int32_t n_planes, const float* const* src,
                         float* const* dst, const int64_t* seg_begin, int32_t n_seg, int64_t* seg_out,
                         int64_t* n_out, char* ws, hipStream_t);
size_t mlp_ws_bytes(int64_t P);
gs_status launch_mlp_features(gs_ctx*, const ViewTab&, const gs_image*, const gs_target*, const gs_mp_frame*, float*,
                              hipStream_t);
gs_status launch_mlp_sync(gs_ctx*, gs_mlp*, hipStream_t);
gs_status launch_mlp_fwd(gs_ctx*, const gs_mlp*, const float*, float*, int64_t, hipStream_t);
gs_status launch_mlp_train(gs_ctx*, gs_mlp*, const float*, const float*, int64_t, float, int, float*, float*, char*,
                           hipStream_t);
