// gs_render_fwd and the per-tile part of gs_render_bwd.
//
// One workgroup of 256 threads per 16x16 tile, one pixel per thread. The
// tile's list is streamed through LDS in batches of records (12 floats each,
// read by all pixels as broadcasts). Forward: front-to-back compositing with
// early exit once every pixel of the tile has stopped. Backward: the same list
// walked back to front from each pixel's n_last, the transmittance recovered
// by dividing by (1 - alpha) from T_final, per-entry gradients summed over the
// wave with DPP, over the 4 waves in LDS, then one atomic per (Gaussian, tile,
// component).
#include "gs_project_dev.h"

namespace {

struct TileCtx {
  int v, tx, ty, px, py;
  bool inside;
  int64_t pix;  // global pixel index (valid when inside)
};

__device__ __forceinline__ TileCtx tile_ctx(const ViewTab& tab, int t) {
  TileCtx c;
  c.v = view_of_tile(tab, t);
  const int lt = t - tab.tile_base[c.v];
  const int gx = tab.gx[c.v];
  c.ty = lt / gx;
  c.tx = lt - c.ty * gx;
  c.px = c.tx * GS_TILE + (threadIdx.x & 15);
  c.py = c.ty * GS_TILE + (threadIdx.x >> 4);
  c.inside = c.px < tab.W[c.v] && c.py < tab.H[c.v];
  c.pix = tab.px_off[c.v] + (int64_t)c.py * tab.W[c.v] + c.px;
  return c;
}

template <int BATCH>
__global__ __launch_bounds__(GS_BLOCK) void render_fwd_kernel(
    ViewTab tab, const float4* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ tile_start, const int32_t* __restrict__ overflow, const int32_t* __restrict__ trunc,
    float bg0, float bg1, float bg2, float* __restrict__ outC, float* __restrict__ outD, float* __restrict__ outM,
    float* __restrict__ outT, uint32_t* __restrict__ nlast, int32_t* __restrict__ incomplete, int truncated_bits) {
  __shared__ float4 s_a[BATCH], s_b[BATCH], s_c[BATCH];
  if (*overflow) return;
  const int t = blockIdx.x;
  const TileCtx tc = tile_ctx(tab, t);
  const uint32_t b = tile_start[t], e = tile_start[t + 1];
  const int64_t roff = tab.r_off[tc.v];
  const float fx = (float)tc.px, fy = (float)tc.py;
  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, Mm = 0.f;
  uint32_t last = 0;
  bool done = !tc.inside;
  bool exhausted = true;
  for (uint32_t base = b; base < e; base += BATCH) {
    if (__syncthreads_count(!done) == 0) {
      exhausted = false;
      break;
    }
    if (threadIdx.x < BATCH && base + threadIdx.x < e) {
      const int64_t r = roff + ids[base + threadIdx.x];
      s_a[threadIdx.x] = rec[3 * r + 0];
      s_b[threadIdx.x] = rec[3 * r + 1];
      s_c[threadIdx.x] = rec[3 * r + 2];
    }
    __syncthreads();
    if (!done) {
      const int n = (int)min((uint32_t)BATCH, e - base);
      for (int j = 0; j < n; ++j) {
        const float4 A = s_a[j];
        const float4 B = s_b[j];
        const float p = gs_power(B.x, B.y, B.z, A.x - fx, A.y - fy);
        if (p > 0.f) continue;
        const float alpha = fminf(GS_ALPHA_MAX, A.w * __expf(p));
        if (alpha < GS_ALPHA_MIN) continue;
        const float Tn = T * (1.0f - alpha);
        if (Tn < GS_T_MIN) {
          done = true;
          break;
        }
        const float4 Cc = s_c[j];
        const float wgt = alpha * T;
        C0 += wgt * Cc.x;
        C1 += wgt * Cc.y;
        C2 += wgt * Cc.z;
        D += wgt * A.z;
        Mm += wgt * B.w;
        T = Tn;
        last = base - b + j + 1;
      }
    }
  }
  // a truncated list ran out while some pixel still lets light through
  if ((truncated_bits >> tc.v) & 1) {
    const int active = __syncthreads_count(!done);
    if (exhausted && active > 0 && threadIdx.x == 0) atomicOr(incomplete, 1);
  }
  if (tc.inside) {
    const int64_t P = tab.npix;
    outC[tc.pix] = C0 + T * bg0;
    outC[P + tc.pix] = C1 + T * bg1;
    outC[2 * P + tc.pix] = C2 + T * bg2;
    outD[tc.pix] = D;
    outM[tc.pix] = Mm;
    outT[tc.pix] = T;
    nlast[tc.pix] = last;
  }
  (void)trunc;
}

// Backward over one tile. g2d is planar [10][nrec]:
// (u_x, u_y, k1, k2, k3, opacity, c_r, c_g, c_b, depth).
template <int BATCH>
__global__ __launch_bounds__(GS_BLOCK) void render_bwd_kernel(
    ViewTab tab, const float4* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ tile_start, const int32_t* __restrict__ overflow, float bg0, float bg1, float bg2,
    const float* __restrict__ imgT, const uint32_t* __restrict__ nlast, const float* __restrict__ dC,
    const float* __restrict__ dD, const float* __restrict__ dM, const float* __restrict__ dT,
    float* __restrict__ g2d, uint8_t* __restrict__ touched) {
  __shared__ float4 s_a[BATCH], s_b[BATCH], s_c[BATCH];
  __shared__ float s_red[BATCH][4][10];
  __shared__ uint32_t s_r[BATCH];
  __shared__ uint32_t s_max;
  if (*overflow) return;
  const int t = blockIdx.x;
  const TileCtx tc = tile_ctx(tab, t);
  const uint32_t b = tile_start[t];
  const int64_t roff = tab.r_off[tc.v];
  const int64_t P = tab.npix;
  const int64_t M = tab.nrec;
  const int w = threadIdx.x >> 6, lane = __lane_id();
  const float fx = (float)tc.px, fy = (float)tc.py;
  float T = 1.f, gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gd = 0.f, gm = 0.f, Tbar = 0.f;
  uint32_t nl = 0;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  if (tc.inside) {
    T = imgT[tc.pix];
    nl = nlast[tc.pix];
    gc0 = dC[tc.pix];
    gc1 = dC[P + tc.pix];
    gc2 = dC[2 * P + tc.pix];
    gd = dD[tc.pix];
    gm = dM ? dM[tc.pix] : 0.f;
    const float gt = dT ? dT[tc.pix] : 0.f;
    Tbar = gt + gc0 * bg0 + gc1 * bg1 + gc2 * bg2;
    atomicMax(&s_max, nl);
  }
  __syncthreads();
  const uint32_t maxl = s_max;
  for (int hi = (int)maxl; hi > 0; hi -= BATCH) {
    const int lo = max(0, hi - BATCH);
    const int n = hi - lo;
    __syncthreads();
    if ((int)threadIdx.x < n) {
      const uint32_t r = (uint32_t)(roff + ids[b + lo + threadIdx.x]);
      s_r[threadIdx.x] = r;
      s_a[threadIdx.x] = rec[3 * (int64_t)r + 0];
      s_b[threadIdx.x] = rec[3 * (int64_t)r + 1];
      s_c[threadIdx.x] = rec[3 * (int64_t)r + 2];
    }
    __syncthreads();
    for (int jj = n - 1; jj >= 0; --jj) {
      const int j = lo + jj;
      float g[10];
#pragma unroll
      for (int c = 0; c < 10; ++c) g[c] = 0.f;
      bool contrib = false;
      if ((uint32_t)j < nl) {
        const float4 A = s_a[jj];
        const float4 B = s_b[jj];
        const float dx = A.x - fx, dy = A.y - fy;
        const float p = gs_power(B.x, B.y, B.z, dx, dy);
        if (p <= 0.f) {
          const float G = __expf(p);
          const float araw = A.w * G;
          const float alpha = fminf(GS_ALPHA_MAX, araw);
          if (alpha >= GS_ALPHA_MIN) {
            contrib = true;
            const float4 Cc = s_c[jj];
            const float one_m = 1.0f - alpha;
            const float Tj = T / one_m;
            const float vdot = gc0 * Cc.x + gc1 * Cc.y + gc2 * Cc.z + gd * A.z + gm * B.w;
            const float abar = Tj * (vdot - Tbar);
            const float wgt = alpha * Tj;
            g[6] = wgt * gc0;
            g[7] = wgt * gc1;
            g[8] = wgt * gc2;
            g[9] = wgt * gd;
            Tbar = vdot * alpha + Tbar * one_m;
            T = Tj;
            if (araw < GS_ALPHA_MAX) {
              const float pbar = abar * alpha;
              g[0] = pbar * (-B.x * dx - B.y * dy);
              g[1] = pbar * (-B.z * dy - B.y * dx);
              g[2] = -0.5f * pbar * dx * dx;
              g[3] = -pbar * dx * dy;
              g[4] = -0.5f * pbar * dy * dy;
              g[5] = abar * G;
            }
          }
        }
      }
      const uint64_t any = __ballot(contrib);
      if (any) {
#pragma unroll
        for (int c = 0; c < 10; ++c) g[c] = wave_sum_to_lane63(g[c]);
      }
      if (lane == 63) {
#pragma unroll
        for (int c = 0; c < 10; ++c) s_red[jj][w][c] = any ? g[c] : 0.f;
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n * 10; q += GS_BLOCK) {
      const int jj = q / 10, c = q - jj * 10;
      const float s = s_red[jj][0][c] + s_red[jj][1][c] + s_red[jj][2][c] + s_red[jj][3][c];
      if (s != 0.f) {
        const uint32_t r = s_r[jj];
        atomicAdd(&g2d[(int64_t)c * M + r], s);
        touched[r] = 1;
      }
    }
  }
}

}  // namespace

gs_status launch_render_fwd(gs_ctx* ctx, const ViewTab& tab, const gs_proj* proj, const gs_bins* bins,
                            const float* bg, int truncated_bits, gs_image* img, hipStream_t s) {
  if (tab.ntiles == 0) return GS_OK;
  const dim3 grid(tab.ntiles), block(GS_BLOCK);
  const float4* rec = (const float4*)proj->rec;
#define GS_FWD(BATCH)                                                                                         \
  GS_LAUNCH(ctx, render_fwd_kernel<BATCH>, grid, block, 0, s, tab, rec, bins->gauss_id, bins->tile_start,      \
                     bins->overflow, nullptr, bg[0], bg[1], bg[2], img->color, img->depth, img->mp, img->T,   \
                     img->n_last, bins->incomplete, truncated_bits)
  switch (ctx->render_batch) {
    case 64: GS_FWD(64); break;
    case 128: GS_FWD(128); break;
    default: GS_FWD(256); break;
  }
#undef GS_FWD
  return gs_check_launch(ctx, "render_fwd");
}

gs_status launch_render_bwd_tiles(gs_ctx* ctx, const ViewTab& tab, const gs_proj* proj, const gs_bins* bins,
                                  const gs_image* img, const gs_pixel_grads* pg, const float* bg, float* g2d,
                                  uint8_t* touched, hipStream_t s) {
  if (tab.ntiles == 0) return GS_OK;
  const dim3 grid(tab.ntiles), block(GS_BLOCK);
  const float4* rec = (const float4*)proj->rec;
#define GS_BWD(BATCH)                                                                                          \
  GS_LAUNCH(ctx, render_bwd_kernel<BATCH>, grid, block, 0, s, tab, rec, bins->gauss_id, bins->tile_start,      \
                     bins->overflow, bg[0], bg[1], bg[2], img->T, img->n_last, pg->dcolor, pg->ddepth, pg->dmp, \
                     pg->dT, g2d, touched)
  switch (ctx->bwd_batch) {
    case 32: GS_BWD(32); break;
    case 128: GS_BWD(128); break;
    default: GS_BWD(64); break;
  }
#undef GS_BWD
  return gs_check_launch(ctx, "render_bwd");
}
