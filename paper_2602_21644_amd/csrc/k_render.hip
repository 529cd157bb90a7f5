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

// Which of a tile's four 16x4 pixel strips (wave w: rows 4w .. 4w+3) an entry
// can composite in: bit w clear only when no pixel of the strip reaches
// alpha >= 1/255. The region where o 2^p >= 1/255, p = c1 dx^2 + c2 dx dy +
// c3 dy^2 (the record's base-2 conic, d = mean - pixel), is the ellipse
// Q <= tau with Q = -p = a dx^2 + b dx dy + c dy^2, (a, b, c) = -(c1, c2, c3),
// and tau = log2(255 o); D = 4ac - b^2. Its half-widths are
// rx = sqrt(4 c tau / D) and ry = sqrt(4 a tau / D). For fixed dx the ellipse
// spans dy = (-b dx +- sqrt(4 c tau - D dx^2)) / (2c); the upper branch is
// concave with its top (dy = ry) at dx = -b ry / (2a), the lower convex with
// its bottom at the opposite dx. So over the tile's columns (dx in an
// interval, cut to |dx| <= rx) the ellipse's rows run from the lower branch at
// the bottom point's dx clamped into the interval to the upper branch at the
// top point's dx clamped into it. The strips that range meets are kept. The
// column interval and the row range are widened by 0.1% of the half-width
// and one pixel against rounding; degenerate or non-finite cases keep every
// strip, o < 1/255 none.
__device__ __forceinline__ uint32_t strip_mask(const float4& A, const float4& B, int x0, int y0) {
  const float tau = __log2f(255.0f * A.w);
  if (tau < 0.f) return 0u;
  const float a = -B.x, bq = -B.y, c = -B.z;
  const float D = 4.0f * a * c - bq * bq;
  if (!(D > 0.f) || !(a > 0.f) || !(c > 0.f) || !(tau < 1e30f)) return 0xFu;
  const float rx = sqrtf(4.0f * c * tau / D), ry = sqrtf(4.0f * a * tau / D);
  if (!(rx < 1e30f) || !(ry < 1e30f) || !(fabsf(A.x) < 1e30f) || !(fabsf(A.y) < 1e30f)) return 0xFu;
  const float mx = 0.001f * rx + 1.0f, my = 0.001f * ry + 1.0f;
  const float dl = fmaxf(A.x - (float)(x0 + 15) - mx, -rx), dh = fminf(A.x - (float)x0 + mx, rx);
  if (dl > dh) return 0u;
  const float dxt = -bq * ry / (2.0f * a);
  const float et = fminf(fmaxf(dxt, dl), dh), eb = fminf(fmaxf(-dxt, dl), dh);
  const float st = sqrtf(fmaxf(0.f, 4.0f * c * tau - D * et * et));
  const float sb = sqrtf(fmaxf(0.f, 4.0f * c * tau - D * eb * eb));
  const float i2c = 0.5f / c;
  const float ylo = A.y - (-bq * et + st) * i2c - my, yhi = A.y - (-bq * eb - sb) * i2c + my;
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float ya = (float)(y0 + 4 * w), yb = (float)(y0 + 4 * w + 3);
    if (!(yhi < ya || ylo > yb)) m |= 1u << w;
  }
  return m;
}

template <int BATCH>
__global__ __launch_bounds__(GS_BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void render_fwd_kernel(
    ViewTab tab, const float4* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ tile_start, const int32_t* __restrict__ overflow, const int32_t* __restrict__ trunc,
    float bg0, float bg1, float bg2, float* __restrict__ outC, float* __restrict__ outD, float* __restrict__ outM,
    float* __restrict__ outT, uint32_t* __restrict__ nlast, uint32_t* __restrict__ tile_work,
    int32_t* __restrict__ incomplete, int32_t* __restrict__ sticky, int cull, LossArgs la) {
  // slot BATCH is a zero-opacity entry that pads a wave's last group of four
  __shared__ float4 s_a[BATCH + 1], s_b[BATCH + 1], s_c[BATCH + 1];
  __shared__ uint8_t s_mask[BATCH];
  // per wave: byte offsets of the batch entries whose mask has the wave's
  // strip, in list order, padded to a multiple of four with the zero entry
  __shared__ __align__(16) uint32_t s_list[GS_BLOCK / 64][BATCH + 4];
  static_assert(BATCH % 4 == 0, "list rows stay 16-byte aligned");
  __shared__ uint32_t s_wmax[GS_BLOCK / 64];
  __shared__ double s_loss[GS_BLOCK / 64];
  if (*overflow) {
    // no image this time; the loss partials still hold a defined value
    if (la.Cg && threadIdx.x == 0) la.part[blockIdx.x] = 0.0;
    return;
  }
  // Launch order: the one the last gs_render_bwd dealt for this tile count
  // (second half of the scheduling state, valid while its marker matches),
  // else the natural order. Any stored order is a permutation of the tiles.
  int t = blockIdx.x;
  if (tile_work) {
    const uint32_t ntl = (uint32_t)tab.ntiles;
    const uint32_t mark = tile_work[2 * (int64_t)ntl], cand = tile_work[ntl + blockIdx.x];
    if (mark == ntl + 1u && cand < ntl) t = (int)cand;
  }
  const TileCtx tc = tile_ctx(tab, t);
  const int w = threadIdx.x >> 6, lane = __lane_id();
  if (threadIdx.x == 0) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    s_a[BATCH] = z;
    s_b[BATCH] = z;
    s_c[BATCH] = z;
  }
  const uint32_t b = tile_start[t], e = tile_start[t + 1];
  const int64_t roff = tab.r_off[tc.v];
  const float fx = (float)tc.px, fy = (float)tc.py;
  // with the loss fused in, the pixel's targets are loaded while it composites
  float tg0 = 0.f, tg1 = 0.f, tg2 = 0.f, tgd = 0.f;
  if (la.Cg && tc.inside) {
    const int64_t P = tab.npix;
    tg0 = la.Cg[tc.pix];
    tg1 = la.Cg[P + tc.pix];
    tg2 = la.Cg[2 * P + tc.pix];
    tgd = la.Dg[tc.pix];
  }
  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, Mm = 0.f;
  uint32_t last = 0;
  uint32_t walked = 0;  // entries this wave evaluated (uniform over the wave)
  bool done = !tc.inside;
  bool exhausted = true;
  // Software pipeline: while a batch is composited, the loader threads hold
  // the next batch's records and the ids of the one after in registers, so
  // neither global load sits between the barriers. Entries past the list
  // end are zero-opacity padding, which never composites.
  const bool loader = threadIdx.x < BATCH;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 ra = z4, rb = z4, rc = z4;
  uint32_t idn = 0;
  if (loader) {
    if (b + threadIdx.x < e) {
      const int64_t r = roff + ids[b + threadIdx.x];
      ra = rec[3 * r + 0];
      rb = rec[3 * r + 1];
      rc = rec[3 * r + 2];
    }
    if (b + BATCH + threadIdx.x < e) idn = ids[b + BATCH + threadIdx.x];
  }
  for (uint32_t base = b; base < e; base += BATCH) {
    if (__syncthreads_count(!done) == 0) {
      exhausted = false;
      break;
    }
    if (loader) {
      s_a[threadIdx.x] = ra;
      s_b[threadIdx.x] = rb;
      s_c[threadIdx.x] = rc;
      s_mask[threadIdx.x] = base + threadIdx.x >= e ? 0u
                            : cull ? (uint8_t)strip_mask(ra, rb, tc.tx * GS_TILE, tc.ty * GS_TILE)
                                   : (uint8_t)0xF;
    }
    __syncthreads();
    if (loader) {
      const uint32_t p1 = base + BATCH + threadIdx.x;
      ra = rb = rc = z4;
      if (p1 < e) {
        const int64_t r = roff + idn;
        ra = rec[3 * r + 0];
        rb = rec[3 * r + 1];
        rc = rec[3 * r + 2];
      }
      if (p1 + BATCH < e) idn = ids[p1 + BATCH];
    }
    if (__any(!done)) {  // uniform over the wave
      const int n = (int)min((uint32_t)BATCH, e - base);
      const uint32_t idx0 = base - b + 1;
      // The wave walks only the entries whose mask has its strip, in list
      // order: it first compacts their LDS offsets into its own list (a
      // ballot per 64 entries), then takes them four at a time, branch-free
      // per entry (every lane evaluates, the predicates select), the early
      // exit tested once per group of four.
      uint32_t* lst = s_list[w];
      int cnt = 0;
      for (int c0 = 0; c0 < n; c0 += 64) {
        const int jl = c0 + lane;
        const bool mine = jl < n && ((s_mask[jl < BATCH ? jl : 0] >> w) & 1u);
        const uint64_t ball = __ballot(mine);
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(ball >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0u));
        if (mine) lst[cnt + below] = (uint32_t)jl * (uint32_t)sizeof(float4);
        cnt += __popcll(ball);
      }
      const int cnt4 = (cnt + 3) & ~3;
      if (lane < cnt4 - cnt) lst[cnt + lane] = (uint32_t)BATCH * (uint32_t)sizeof(float4);
      __builtin_amdgcn_wave_barrier();
      const char* pa = reinterpret_cast<const char*>(s_a);
      const char* pb = reinterpret_cast<const char*>(s_b);
      const char* pc = reinterpret_cast<const char*>(s_c);
      int k = 0;
      for (; k < cnt4; k += 4) {
        const uint4 o4 = *reinterpret_cast<const uint4*>(&lst[k]);
        const uint32_t os[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float4 A = *reinterpret_cast<const float4*>(pa + os[u]);
          const float4 B = *reinterpret_cast<const float4*>(pb + os[u]);
          const float4 Cc = *reinterpret_cast<const float4*>(pc + os[u]);
          const float p = gs_power2(B.x, B.y, B.z, A.x - fx, A.y - fy);
          const float alpha = fminf(GS_ALPHA_MAX, A.w * __builtin_amdgcn_exp2f(p));
          const bool ok = !done && p <= 0.f && alpha >= GS_ALPHA_MIN;
          const float Tn = T * (1.0f - alpha);
          const bool stop = ok && Tn < GS_T_MIN;
          const bool add = ok != stop;  // ok and not stop (stop implies ok)
          done = done || stop;
          const float wgt = add ? alpha * T : 0.f;
          C0 += wgt * Cc.x;
          C1 += wgt * Cc.y;
          C2 += wgt * Cc.z;
          D += wgt * A.z;
          Mm += wgt * B.w;
          T = add ? Tn : T;
          last = add ? idx0 + os[u] / (uint32_t)sizeof(float4) : last;
        }
        if (__all(done)) {
          k += 4;
          break;
        }
      }
      walked += (uint32_t)k;
    }
  }
  // a list that leaves out visible records ran out while some pixel still
  // lets light through
  if (trunc && ((*trunc >> tc.v) & 1)) {
    const int active = __syncthreads_count(!done);
    if (exhausted && active > 0 && threadIdx.x == 0) {
      atomicOr(incomplete, 1);
      if (sticky) atomicOr(&sticky[1], 1);
    }
  }
  double lsum = 0.0;
  if (tc.inside) {
    const int64_t P = tab.npix;
    const float c0 = C0 + T * bg0, c1 = C1 + T * bg1, c2 = C2 + T * bg2;
    outC[tc.pix] = c0;
    outC[P + tc.pix] = c1;
    outC[2 * P + tc.pix] = c2;
    outD[tc.pix] = D;
    outM[tc.pix] = Mm;
    outT[tc.pix] = T;
    nlast[tc.pix] = last;
    if (la.Cg) lsum = pixel_loss(la, P, tc.pix, c0, c1, c2, D, Mm, T, tg0, tg1, tg2, tgd);
  }
  if (tile_work || la.Cg) {
    // the tile's work: the entries its four waves evaluated; the tile's loss
    // partial
    if (la.Cg) lsum = wave_sum_all_d(lsum);
    if (lane == 0) s_wmax[w] = walked;
    if (lane == 63) s_loss[w] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t sum = 0;
#pragma unroll
      for (int i = 0; i < GS_BLOCK / 64; ++i) sum += s_wmax[i];
      if (tile_work) tile_work[t] = sum;
      if (la.Cg) la.part[t] = s_loss[0] + s_loss[1] + s_loss[2] + s_loss[3];
    }
  }
}

// Launch order of the backward's tiles, heaviest first by tile_work: a
// counting sort into log-scale buckets (16 per octave, from the float32 bits
// of the work), then rank r goes to block round * n_cu + (round even ? i :
// m - 1 - i) with round = r / n_cu, i = r mod n_cu and m the blocks of that
// round. While the whole grid is resident, blocks b and b + n_cu share a
// compute unit, so this snake deal evens the work per unit; with more blocks
// than fit, the heaviest tiles still start first. order[b] is the tile block b
// runs; every tile appears once; order[n] = n + 1 marks it complete.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 2048;
constexpr int kOrderCached = 16384;  // tiles whose buckets stay in LDS
__device__ __forceinline__ int order_bucket(uint32_t x) {
  const int k = (int)(__float_as_uint((float)x) >> 19) - (127 << 4) + 1;  // x = 0 -> below 0, x = 1 -> 1
  return kOrderBuckets - 1 - min(max(k, 0), kOrderBuckets - 1);
}
__device__ void deal_tile_order(const uint32_t* __restrict__ work, int ntiles, int ncu,
                                uint32_t* __restrict__ order) {
  __shared__ uint32_t s_cnt[kOrderBuckets];
  __shared__ uint16_t s_bk[kOrderCached];
  __shared__ uint32_t s_wave[kOrderThreads / 64];
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  const bool cached = ntiles <= kOrderCached;
  for (int i = tid; i < kOrderBuckets; i += kOrderThreads) s_cnt[i] = 0;
  __syncthreads();
  for (int t = tid; t < ntiles; t += kOrderThreads) {
    const int bk = order_bucket(work[t]);
    if (cached) s_bk[t] = (uint16_t)bk;
    atomicAdd(&s_cnt[bk], 1u);
  }
  __syncthreads();
  // exclusive scan of the buckets, two per thread
  const uint32_t c0 = s_cnt[2 * tid], c1 = s_cnt[2 * tid + 1];
  uint32_t incl = c0 + c1;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_wave[wv] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (int i = 0; i < wv; ++i) before += s_wave[i];
  const uint32_t ex = before + incl - (c0 + c1);
  s_cnt[2 * tid] = ex;
  s_cnt[2 * tid + 1] = ex + c0;
  __syncthreads();
  const uint32_t n = (uint32_t)ntiles, c = (uint32_t)max(ncu, 1);
  for (int t = tid; t < ntiles; t += kOrderThreads) {
    const int bk = cached ? (int)s_bk[t] : order_bucket(work[t]);
    const uint32_t r = atomicAdd(&s_cnt[bk], 1u);
    if (r >= n) continue;  // never taken: the ranks are 0 .. n - 1
    const uint32_t k = r / c, i = r - k * c;
    const uint32_t mk = min(c, n - k * c);
    order[k * c + ((k & 1) ? mk - 1 - i : i)] = (uint32_t)t;
  }
  if (tid == 0) order[n] = n + 1u;  // marks the order valid for n tiles
}

__global__ __launch_bounds__(kOrderThreads) void tile_order_kernel(const uint32_t* __restrict__ work, int ntiles,
                                                                   int ncu, uint32_t* __restrict__ order) {
  deal_tile_order(work, ntiles, ncu, order);
}

// After the forward with the loss fused in: workgroup v < nv sums view v's
// per-tile loss partials in a fixed order (float64); one more workgroup, when
// `order` is set, deals the tile order as tile_order_kernel does.
__global__ __launch_bounds__(kOrderThreads) void fwd_finish_kernel(ViewTab tab, const double* __restrict__ part,
                                                                   float* __restrict__ loss,
                                                                   const uint32_t* __restrict__ work, int ncu,
                                                                   uint32_t* __restrict__ order) {
  if ((int)blockIdx.x >= tab.nv) {
    deal_tile_order(work, tab.ntiles, ncu, order);
    return;
  }
  __shared__ double s_sum[kOrderThreads / 64];
  const int v = blockIdx.x;
  const int nt = tab.gx[v] * tab.gy[v];
  const double* pv = part + tab.tile_base[v];
  constexpr int kU = 4;
  double acc = 0.0;
  for (int b0 = threadIdx.x; b0 < nt; b0 += kU * kOrderThreads) {
    double x[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = b0 + u * kOrderThreads < nt ? pv[b0 + u * kOrderThreads] : 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u) acc += x[u];
  }
  acc = wave_sum_all_d(acc);
  if (__lane_id() == 63) s_sum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kOrderThreads / 64; ++i) t += s_sum[i];
    loss[v] = (float)t;
  }
}

// Backward over one tile. g2d holds per record ten values
// (u_x, u_y, k1, k2, k3, opacity, c_r, c_g, c_b, depth), [copy][record][10].
//
// Per entry every lane forms ten moment terms of its pixel, with
// h = dL/d(alpha) * exp(power) where alpha is unclamped, else 0:
//   h*dx, h*dy, h*dx^2, h*dx*dy, h*dy^2, h, w*gC (3), w*gD   (w = alpha*T)
// A transposed wave reduction sums them; the cross-wave pass turns the sums
// into the 2D gradients with the entry's opacity and conic
// (d/du = -o * conic * (sum h*d), d/dconic = -o/2 * (sum h*d d^T) off-diagonal
// counted twice), so the per-pixel work carries no conic products.
// The dense gradient outputs, zeroed by the tile pass: workgroup b clears
// Gaussians [b chunk, (b + 1) chunk) of all fourteen planes once its tile is
// done, so the stores overlap the other workgroups' compositing; the
// projection adjoint then writes the listed Gaussians over the zeros.
struct GradZero {
  float* plane[14];  // NULL first plane: nothing to clear (pose only, or accumulating)
  int64_t n, chunk;  // chunk: a multiple of 4
  int vec4;          // n % 4 == 0 and every plane 16-byte aligned
};

__device__ __forceinline__ void zero_grad_slice(const GradZero& z, int blk) {
  if (!z.plane[0]) return;
  const int64_t lo = (int64_t)blk * z.chunk, hi = min(lo + z.chunk, z.n);
  if (z.vec4) {
    for (int64_t i = (lo >> 2) + threadIdx.x; i < (hi >> 2); i += GS_BLOCK)
#pragma unroll
      for (int q = 0; q < 14; ++q) reinterpret_cast<float4*>(z.plane[q])[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    for (int64_t k = lo + threadIdx.x; k < hi; k += GS_BLOCK)
#pragma unroll
      for (int q = 0; q < 14; ++q) z.plane[q][k] = 0.f;
  }
}

template <int BATCH, bool POSE>
__global__ __launch_bounds__(GS_BLOCK) __attribute__((amdgpu_waves_per_eu(5))) void render_bwd_kernel(
    ViewTab tab, const float4* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ tile_start, const int32_t* __restrict__ overflow, float bg0, float bg1, float bg2,
    const float* __restrict__ imgT, const uint32_t* __restrict__ nlast, const float* __restrict__ dC,
    const float* __restrict__ dD, const float* __restrict__ dM, const float* __restrict__ dT,
    const float* __restrict__ vw, float* __restrict__ g2d, TouchArgs touch, const uint32_t* __restrict__ order,
    int copies, int cull, GradZero zg) {
  __shared__ float4 s_a[BATCH], s_b[BATCH], s_c[BATCH];
  __shared__ uint8_t s_mask[BATCH];
  // per wave: the batch entries it walks (mask has its strip, inside its
  // longest n_last), in list order
  __shared__ int32_t s_list[GS_BLOCK / 64][BATCH];
  __shared__ uint32_t s_wmax[GS_BLOCK / 64];
  // [entry][wave * 4 + row]: the three row totals of wave_sum10; the 17th
  // slot staggers the entries across LDS banks for the cross-wave pass
  __shared__ float4 s_red[BATCH][17];
  __shared__ uint32_t s_r[BATCH];
  __shared__ uint32_t s_max;
  if (*overflow) {
    zero_grad_slice(zg, blockIdx.x);
    return;
  }
  // the order the forward dealt, while its marker is valid for this tile count
  uint32_t tu = blockIdx.x;
  if (order) {
    const uint32_t ntl = (uint32_t)tab.ntiles, cand = order[blockIdx.x];
    if (order[ntl] == ntl + 1u && cand < ntl) tu = cand;
  }
  const int t = (int)tu;
  const TileCtx tc = tile_ctx(tab, t);
  const uint32_t b = tile_start[t];
  const int64_t roff = tab.r_off[tc.v];
  const int64_t P = tab.npix;
  const int64_t M = tab.nrec;
  const int w = threadIdx.x >> 6, lane = __lane_id();
  // The 2D adjoint has `copies` accumulators; a workgroup adds into the one of
  // the XCD it runs on (hardware register XCC_ID). The sums do not depend on
  // the split; it keeps the atomics of the XCDs on a record apart, which
  // would otherwise contend for the same addresses.
  // Layout [copy][record][10].
  if (copies > 1) g2d += (int64_t)(__builtin_amdgcn_s_getreg((31 << 11) | 20) & (uint32_t)(copies - 1)) * 10 * M;
  const float fx = (float)tc.px, fy = (float)tc.py;
  float T = 1.f, gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gd = 0.f, gm = 0.f, Tbar = 0.f;
  uint32_t nl = 0;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  if (tc.inside) {
    T = imgT[tc.pix];
    nl = nlast[tc.pix];
    // the view's loss weight scales all of its pixel adjoints
    const float sw = vw ? vw[tc.v] : 1.f;
    gc0 = dC[tc.pix] * sw;
    gc1 = dC[P + tc.pix] * sw;
    gc2 = dC[2 * P + tc.pix] * sw;
    gd = dD[tc.pix] * sw;
    gm = dM ? dM[tc.pix] * sw : 0.f;
    const float gt = dT ? dT[tc.pix] * sw : 0.f;
    Tbar = gt + gc0 * bg0 + gc1 * bg1 + gc2 * bg2;
  }
  // longest list prefix any pixel of this wave composited
  uint32_t wmax = nl;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, o, 64));
  if (lane == 0) {
    atomicMax(&s_max, wmax);
    s_wmax[w] = wmax;
  }
  __syncthreads();
  const uint32_t maxl = s_max;
  // Batches walk back: [lo, hi) with hi = maxl, then hi = previous lo. As in
  // the forward, the next batch's records and the ids of the one after are
  // loaded into registers while a batch is processed.
  const int tid = (int)threadIdx.x;
  float4 ra, rb, rc;
  uint32_t rn = 0, idn = 0;
  {
    const int lo0 = max(0, (int)maxl - BATCH), lo1 = max(0, lo0 - BATCH);
    if (tid < (int)maxl - lo0) {
      rn = (uint32_t)(roff + ids[b + lo0 + tid]);
      ra = rec[3 * (int64_t)rn + 0];
      rb = rec[3 * (int64_t)rn + 1];
      rc = rec[3 * (int64_t)rn + 2];
    }
    if (tid < lo0 - lo1) idn = ids[b + lo1 + tid];
  }
  for (int hi = (int)maxl; hi > 0; hi -= BATCH) {
    const int lo = max(0, hi - BATCH);
    const int n = hi - lo;
    __syncthreads();
    if (tid < n) {
      s_r[tid] = rn;
      s_a[tid] = ra;
      s_b[tid] = rb;
      s_c[tid] = rc;
      s_mask[tid] = cull ? (uint8_t)strip_mask(ra, rb, tc.tx * GS_TILE, tc.ty * GS_TILE) : (uint8_t)0xF;
    }
    __syncthreads();
    {
      const int lo1 = max(0, lo - BATCH), lo2 = max(0, lo1 - BATCH);
      if (tid < lo - lo1) {
        rn = (uint32_t)(roff + idn);
        ra = rec[3 * (int64_t)rn + 0];
        rb = rec[3 * (int64_t)rn + 1];
        rc = rec[3 * (int64_t)rn + 2];
      }
      if (tid < lo1 - lo2) idn = ids[b + lo2 + tid];
    }
    // One entry of the batch; two register sets alternate below so that the
    // next entry's record is read from LDS while this one is processed.
    auto entry = [&](int jj, const float4& A, const float4& B) {
      const int j = lo + jj;
      float k[3] = {0.f, 0.f, 0.f};
      {
        const float dx = A.x - fx, dy = A.y - fy;
        const float p = gs_power2(B.x, B.y, B.z, dx, dy);
        const float G = __builtin_amdgcn_exp2f(p);
        const float araw = A.w * G;
        const float alpha = fminf(GS_ALPHA_MAX, araw);
        const bool valid = (uint32_t)j < nl && p <= 0.f && alpha >= GS_ALPHA_MIN;
        if (__ballot(valid)) {  // uniform
          const float4 Cc = s_c[jj];  // colour only for entries some pixel composites
          const float a = valid ? alpha : 0.f;
          const float one_m = 1.0f - a;
          const float Tj = T * __builtin_amdgcn_rcpf(one_m);
          const float vdot = gc0 * Cc.x + gc1 * Cc.y + gc2 * Cc.z + gd * A.z + gm * B.w;
          const float abar = Tj * (vdot - Tbar);
          const float wgt = a * Tj;
          const float h = (valid && araw < GS_ALPHA_MAX) ? abar * G : 0.f;
          Tbar = vdot * a + Tbar * one_m;
          T = Tj;
          if constexpr (POSE) {
            // the pose moves the mean, the conic and the depth only
            float v[6];
            v[0] = h * dx;
            v[1] = h * dy;
            v[2] = v[0] * dx;
            v[3] = v[0] * dy;
            v[4] = v[1] * dy;
            v[5] = wgt * gd;
            wave_sum6(v, k);
          } else {
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
      }
      if ((lane & 15) == 15) s_red[jj][w * 4 + (lane >> 4)] = make_float4(k[0], k[1], k[2], 0.f);
    };
    // An entry the wave does not walk has no pixel of the wave with alpha
    // >= 1/255 (its mask misses the strip) or lies past every pixel's n_last:
    // it adds nothing, and the cross-wave pass skips the wave's rows of it.
    // The rest are compacted by a ballot per 64 entries and walked from the
    // back.
    int32_t* lst = s_list[w];
    int cnt = 0;
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int jl = c0 + lane;
      const bool mine = jl < n && (uint32_t)(lo + jl) < wmax && ((s_mask[jl < BATCH ? jl : 0] >> w) & 1u);
      const uint64_t ball = __ballot(mine);
      const int below =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(ball >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0u));
      if (mine) lst[cnt + below] = jl;
      cnt += __popcll(ball);
    }
    __builtin_amdgcn_wave_barrier();
    // the next entry's index is read from the list while one is processed
    int jn = cnt > 0 ? lst[cnt - 1] : 0;
#pragma unroll 1
    for (int kk = cnt - 1; kk >= 0; --kk) {
      const int j0 = jn;
      jn = lst[kk > 0 ? kk - 1 : 0];
      entry(j0, s_a[j0], s_b[j0]);
    }
    __syncthreads();
    // The cross-wave pass runs on the waves that load nothing: one counter
    // tracks both loads and atomics, so the loader waves' wait for the next
    // records never includes this batch's atomics.
    constexpr int kLoadThreads = (BATCH + 63) / 64 * 64;
    static_assert(kLoadThreads < GS_BLOCK, "some wave must be free of loads");
    // one thread per entry: all sixteen row totals in one LDS round trip,
    // then the entry's ten gradient components and their atomics
    static_assert(GS_BLOCK - kLoadThreads >= BATCH, "a thread per entry");
    const int q = tid - kLoadThreads;
    if (q >= 0 && q < n) {
      const int jj = q;
      const uint32_t msk = s_mask[jj];
      float4 rw[4][4];
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        const bool walked = ((msk >> ww) & 1u) && (uint32_t)(lo + jj) < s_wmax[ww];
#pragma unroll
        for (int row = 0; row < 4; ++row)
          rw[ww][row] = walked ? s_red[jj][ww * 4 + row] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      float4 t0 = rw[0][0], t1 = rw[0][1], t2 = rw[0][2], t3 = rw[0][3];
#pragma unroll
      for (int ww = 1; ww < 4; ++ww) {
        t0.x += rw[ww][0].x; t0.y += rw[ww][0].y; t0.z += rw[ww][0].z;
        t1.x += rw[ww][1].x; t1.y += rw[ww][1].y;
        t2.x += rw[ww][2].x; t2.y += rw[ww][2].y; t2.z += rw[ww][2].z;
        t3.x += rw[ww][3].x; t3.y += rw[ww][3].y;
      }
      float m0, m1, m2, m3, m4, m5, m6, m7, m8, m9;
      if constexpr (POSE) {
        // wave_sum6's rows: (m0, m2), (m1, -), (m3, m9), (m4, -); the opacity
        // and colour sums are not formed
        m0 = t0.x; m2 = t0.y; m1 = t1.x; m3 = t2.x; m9 = t2.y; m4 = t3.x;
        m5 = m6 = m7 = m8 = 0.f;
      } else {
        // wave_sum10's rows: (m0, m2, m4), (m1, m3, -), (m5, m7, m9), (m6, m8, -)
        m0 = t0.x; m2 = t0.y; m4 = t0.z; m1 = t1.x; m3 = t1.y;
        m5 = t2.x; m7 = t2.y; m9 = t2.z; m6 = t3.x; m8 = t3.y;
      }
      const float o = s_a[jj].w;
      const float4 B = s_b[jj];
      // back from base-2 exponent units to the conic
      const float k1 = B.x * (-2.0f / GS_LOG2E), k2 = B.y * (-1.0f / GS_LOG2E), k3 = B.z * (-2.0f / GS_LOG2E);
      float gv[10];
      gv[0] = -o * (k1 * m0 + k2 * m1);
      gv[1] = -o * (k2 * m0 + k3 * m1);
      gv[2] = -0.5f * o * m2;
      gv[3] = -o * m3;
      gv[4] = -0.5f * o * m4;
      gv[5] = m5;
      gv[6] = m6;
      gv[7] = m7;
      gv[8] = m8;
      gv[9] = m9;
      // back into the entry's first three slots (this thread read them)
      s_red[jj][0] = make_float4(gv[0], gv[1], gv[2], gv[3]);
      s_red[jj][1] = make_float4(gv[4], gv[5], gv[6], gv[7]);
      s_red[jj][2] = make_float4(gv[8], gv[9], 0.f, 0.f);
      // the first tile that gives a Gaussian a gradient lists it (once per
      // call) for the projection adjoint
      bool any = false;
#pragma unroll
      for (int c = 0; c < 10; ++c) any = any || gv[c] != 0.f;
      if (any) {
        const uint32_t gk = (uint32_t)(tab.g_off[tc.v] + ((int64_t)s_r[jj] - roff));
        if (touch.flag[gk] == 0u && atomicExch(&touch.flag[gk], 1u) == 0u) touch.list[atomicAdd(touch.count, 1u)] = gk;
      }
    }
    __syncthreads();
    // ten adjacent threads per entry: a wave's atomics fall on few lines
    for (int qq = tid - kLoadThreads; qq >= 0 && qq < n * 10; qq += GS_BLOCK - kLoadThreads) {
      const int jj = qq / 10, c = qq - jj * 10;
      const float gval = reinterpret_cast<const float*>(&s_red[jj][0])[c];
      if (gval != 0.f) atomicAdd(&g2d[(int64_t)s_r[jj] * 10 + c], gval);
    }
  }
  zero_grad_slice(zg, blockIdx.x);
}


}  // namespace

// Compute units of the device, queried once per context.
static gs_status query_n_cu(gs_ctx* ctx) {
  if (ctx->n_cu > 0) return GS_OK;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || n <= 0)
    return gs_fail(ctx, GS_E_HIP, "cannot query the compute-unit count");
  ctx->n_cu = n;
  return GS_OK;
}

gs_status launch_render_fwd(gs_ctx* ctx, const ViewTab& tab, const gs_proj* proj, const gs_bins* bins,
                            const float* bg, gs_image* img, hipStream_t s, const LossArgs* loss) {
  if (tab.ntiles == 0) return GS_OK;
  const dim3 grid(tab.ntiles), block(GS_BLOCK);
  const float4* rec = (const float4*)proj->rec;
  LossArgs la{};
  if (loss) la = *loss;
#define GS_FWD(BATCH)                                                                                         \
  GS_LAUNCH(ctx, render_fwd_kernel<BATCH>, grid, block, 0, s, tab, rec, bins->gauss_id, bins->tile_start,      \
                     bins->overflow, bins->max_rank > 0 ? bins->truncated : nullptr, bg[0], bg[1], bg[2],       \
                     img->color, img->depth, img->mp, img->T, img->n_last, img->tile_work, bins->incomplete,   \
                     bins->sticky, ctx->wave_cull, la)
  switch (ctx->render_batch) {
    case 64: GS_FWD(64); break;
    case 128: GS_FWD(128); break;
    default: GS_FWD(256); break;
  }
#undef GS_FWD
  // the backward's tile order (and the per-view loss sums when fused)
  const bool deal = img->tile_work && ctx->tile_order;
  if (deal) {
    const gs_status st = query_n_cu(ctx);
    if (st != GS_OK) return st;
  }
  uint32_t* ord = img->tile_work ? img->tile_work + tab.ntiles : nullptr;
  if (loss)
    GS_LAUNCH(ctx, fwd_finish_kernel, dim3(tab.nv + (deal ? 1 : 0)), dim3(kOrderThreads), 0, s, tab, la.part,
              la.loss, img->tile_work, ctx->n_cu, ord);
  else if (deal)
    GS_LAUNCH(ctx, tile_order_kernel, dim3(1), dim3(kOrderThreads), 0, s, img->tile_work, (int)tab.ntiles,
              ctx->n_cu, ord);
  return gs_check_launch(ctx, "render_fwd");
}

gs_status launch_render_bwd_tiles(gs_ctx* ctx, const ViewTab& tab, const gs_proj* proj, const gs_bins* bins,
                                  const gs_image* img, const gs_pixel_grads* pg, const float* bg, float* g2d,
                                  TouchArgs touch, const gs_grads* gr, hipStream_t s) {
  if (tab.ntiles == 0) return GS_OK;  // the projection adjoint then clears the gradients itself
  const dim3 grid(tab.ntiles), block(GS_BLOCK);
  GradZero zg{};
  if (!gr->pose_only && !gr->accumulate && tab.ng > 0) {
    const int64_t n = tab.ng;
    float* const pl[14] = {gr->mean,          gr->mean + n,      gr->mean + 2 * n, gr->log_scale,
                           gr->log_scale + n, gr->log_scale + 2 * n, gr->quat,     gr->quat + n,
                           gr->quat + 2 * n,  gr->quat + 3 * n,  gr->opacity_logit, gr->color,
                           gr->color + n,     gr->color + 2 * n};
    bool vec4 = (n & 3) == 0;
    for (int q = 0; q < 14; ++q) {
      zg.plane[q] = pl[q];
      vec4 = vec4 && ((uintptr_t)pl[q] & 15) == 0;
    }
    zg.n = n;
    zg.chunk = ((n + tab.ntiles - 1) / tab.ntiles + 3) & ~(int64_t)3;
    zg.vec4 = vec4 ? 1 : 0;
  }
  const float4* rec = (const float4*)proj->rec;
  // the order the last forward dealt (second half of the scheduling state)
  const uint32_t* order = img->tile_work && ctx->tile_order ? img->tile_work + tab.ntiles : nullptr;
#define GS_BWD(BATCH, POSE)                                                                                   \
  GS_LAUNCH_NAMED(ctx, POSE ? "render_bwd_pose_kernel<" #BATCH ">" : "render_bwd_kernel<" #BATCH ">",          \
                  (render_bwd_kernel<BATCH, POSE>), grid, block, 0, s, tab, rec, bins->gauss_id,               \
                  bins->tile_start, bins->overflow, bg[0], bg[1], bg[2], img->T, img->n_last, pg->dcolor,      \
                  pg->ddepth, pg->dmp, pg->dT, pg->view_weight, g2d, touch, order, ctx->bwd_copies,            \
                  ctx->wave_cull, zg)
  const bool pose = gr->pose_only != 0;
  switch (ctx->bwd_batch) {
    case 32: if (pose) GS_BWD(32, true); else GS_BWD(32, false); break;
    case 128: if (pose) GS_BWD(128, true); else GS_BWD(128, false); break;
    default: if (pose) GS_BWD(64, true); else GS_BWD(64, false); break;
  }
#undef GS_BWD
  return gs_check_launch(ctx, "render_bwd");
}
