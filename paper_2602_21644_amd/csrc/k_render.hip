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
    if (threadIdx.x < BATCH) {
      if (base + threadIdx.x < e) {
        const int64_t r = roff + ids[base + threadIdx.x];
        s_a[threadIdx.x] = rec[3 * r + 0];
        s_b[threadIdx.x] = rec[3 * r + 1];
        s_c[threadIdx.x] = rec[3 * r + 2];
      } else {
        // padding: zero opacity never composites
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        s_a[threadIdx.x] = z;
        s_b[threadIdx.x] = z;
        s_c[threadIdx.x] = z;
      }
    }
    __syncthreads();
    if (__any(!done)) {  // uniform over the wave
      const int n = (int)min((uint32_t)BATCH, e - base);
      const uint32_t idx0 = base - b + 1;
      // branch-free per entry: every lane evaluates, the predicates select;
      // groups of four, the early exit tested once per group
      for (int j0 = 0; j0 < n; j0 += 4) {
#pragma unroll
      for (int j = j0; j < j0 + 4; ++j) {
        const float4 A = s_a[j];
        const float4 B = s_b[j];
        const float4 Cc = s_c[j];
        const float p = gs_power(B.x, B.y, B.z, A.x - fx, A.y - fy);
        const float alpha = fminf(GS_ALPHA_MAX, A.w * __expf(p));
        const bool ok = !done && p <= 0.f && alpha >= GS_ALPHA_MIN;
        const float Tn = T * (1.0f - alpha);
        const bool stop = ok && Tn < GS_T_MIN;
        const bool add = ok && !stop;
        done = done || stop;
        const float wgt = add ? alpha * T : 0.f;
        C0 += wgt * Cc.x;
        C1 += wgt * Cc.y;
        C2 += wgt * Cc.z;
        D += wgt * A.z;
        Mm += wgt * B.w;
        T = add ? Tn : T;
        last = add ? idx0 + j : last;
      }
      if (__all(done)) break;
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
//
// Per entry every lane forms ten moment terms of its pixel, with
// h = dL/d(alpha) * exp(power) where alpha is unclamped, else 0:
//   h*dx, h*dy, h*dx^2, h*dx*dy, h*dy^2, h, w*gC (3), w*gD   (w = alpha*T)
// A transposed wave reduction sums them; the cross-wave pass turns the sums
// into the 2D gradients with the entry's opacity and conic
// (d/du = -o * conic * (sum h*d), d/dconic = -o/2 * (sum h*d d^T) off-diagonal
// counted twice), so the per-pixel work carries no conic products.
// Backward over one tile. g2d is planar [10][nrec]:
// (u_x, u_y, k1, k2, k3, opacity, c_r, c_g, c_b, depth).
//
// Per entry every lane forms ten moment terms of its pixel, with
// h = dL/d(alpha) * exp(power) where alpha is unclamped, else 0:
//   h*dx, h*dy, h*dx^2, h*dx*dy, h*dy^2, h, w*gC (3), w*gD   (w = alpha*T)
// A transposed wave reduction sums them; the cross-wave pass turns the sums
// into the 2D gradients with the entry's opacity and conic
// (d/du = -o * conic * (sum h*d), d/dconic = -o/2 * (sum h*d d^T) off-diagonal
// counted twice), so the per-pixel work carries no conic products.
template <int BATCH>
__global__ __launch_bounds__(GS_BLOCK) void render_bwd_kernel(
    ViewTab tab, const float4* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ tile_start, const int32_t* __restrict__ overflow, float bg0, float bg1, float bg2,
    const float* __restrict__ imgT, const uint32_t* __restrict__ nlast, const float* __restrict__ dC,
    const float* __restrict__ dD, const float* __restrict__ dM, const float* __restrict__ dT,
    float* __restrict__ g2d, uint8_t* __restrict__ touched) {
  __shared__ float4 s_a[BATCH], s_b[BATCH], s_c[BATCH];
  __shared__ float4 s_red[BATCH][4][4];  // [entry][wave][row]: the three row totals of wave_sum10
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
  }
  // longest list prefix any pixel of this wave composited
  uint32_t wmax = nl;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, o, 64));
  if (lane == 0) atomicMax(&s_max, wmax);
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
      float k[3] = {0.f, 0.f, 0.f};
      if ((uint32_t)j < wmax) {  // uniform over the wave
        const float4 A = s_a[jj];
        const float4 B = s_b[jj];
        const float4 Cc = s_c[jj];
        const float dx = A.x - fx, dy = A.y - fy;
        const float p = gs_power(B.x, B.y, B.z, dx, dy);
        const float G = __expf(p);
        const float araw = A.w * G;
        const float alpha = fminf(GS_ALPHA_MAX, araw);
        const bool valid = (uint32_t)j < nl && p <= 0.f && alpha >= GS_ALPHA_MIN;
        if (__ballot(valid)) {  // uniform
          const float a = valid ? alpha : 0.f;
          const float one_m = 1.0f - a;
          const float Tj = T * __builtin_amdgcn_rcpf(one_m);
          const float vdot = gc0 * Cc.x + gc1 * Cc.y + gc2 * Cc.z + gd * A.z + gm * B.w;
          const float abar = Tj * (vdot - Tbar);
          const float wgt = a * Tj;
          const float h = (valid && araw < GS_ALPHA_MAX) ? abar * G : 0.f;
          Tbar = vdot * a + Tbar * one_m;
          T = Tj;
          float v[10];
          v[0] = h * dx;
          v[1] = h * dy;
          v[2] = v[0] * dx;
          v[3] = v[0] * dy;
          v[4] = v[1] * dy;
          v[5] = h;
          v[6] = wgt * gc0;
          v[7] = wgt * gc1;
          v[8] = wgt * gc2;
          v[9] = wgt * gd;
          wave_sum10(v, k);
        }
      }
      if ((lane & 15) == 15) s_red[jj][w][lane >> 4] = make_float4(k[0], k[1], k[2], 0.f);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n * 10; q += GS_BLOCK) {
      const int jj = q / 10, c = q - jj * 10;
      // moment index -> (row, slot) of wave_sum10's output
      auto mom = [&](int m) {
        const int row = m < 5 ? (m & 1) : 2 + ((m - 5) & 1);
        const int sl = m < 5 ? (m >> 1) : ((m - 5) >> 1);
        float acc = 0.f;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
          const float4 x = s_red[jj][ww][row];
          acc += sl == 0 ? x.x : (sl == 1 ? x.y : x.z);
        }
        return acc;
      };
      const float o = s_a[jj].w;
      float gval;
      if (c < 2) {
        const float4 B = s_b[jj];
        const float s0 = mom(0), s1 = mom(1);
        gval = c == 0 ? -o * (B.x * s0 + B.y * s1) : -o * (B.y * s0 + B.z * s1);
      } else if (c == 2 || c == 4) {
        gval = -0.5f * o * mom(c);
      } else if (c == 3) {
        gval = -o * mom(3);
      } else {
        gval = mom(c);
      }
      if (gval != 0.f) {
        const uint32_t r = s_r[jj];
        atomicAdd(&g2d[(int64_t)c * M + r], gval);
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
