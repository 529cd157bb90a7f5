// gs_project: coalesced planar reads of the Gaussian parameters, one record
// per thread and pass; writes the tile rect and depth key (plus the key
// histogram and the optional planar outputs). The 48-byte compositing record
// is written here only for full binning; with the prefix path it is written
// by gs_bin_sort for the few records the lists reference.
#include "gs_project_dev.h"

namespace {

constexpr int PBLOCK = 1024;
constexpr int PITEMS = 4;  // records per thread: 4096 per workgroup amortises the histogram

__device__ __forceinline__ uint32_t project_one(const ViewTab& tab, const gs_camera& cam,
                                                const float* __restrict__ mean, const float* __restrict__ log_scale,
                                                const float* __restrict__ quat, const float* __restrict__ opl,
                                                const float* __restrict__ color, const float* __restrict__ mp,
                                                float4* __restrict__ rec, int2* __restrict__ rect,
                                                uint32_t* __restrict__ key,
                                                float* __restrict__ mean2d, float* __restrict__ conic,
                                                float* __restrict__ depth, float* __restrict__ opacity,
                                                int32_t* __restrict__ radius, int v, int64_t k) {
  const int64_t r = tab.r_off[v] + k;
  const int64_t M = tab.nrec;
  const int64_t N = tab.ng;
  // empty rect: x0 = 1 > x1 = 0
  const int2 empty_rect = make_int2((int)(uint16_t)1 | ((int)(uint16_t)1 << 16), 0);
  if (k >= tab.n[v]) {
    rect[r] = empty_rect;
    key[r] = 0xFFFFFFFFu;
    if (radius) radius[r] = 0;
    return 0xFFFFFFFFu;
  }
  const int64_t gk = tab.g_off[v] + k;
  const float m[3] = {mean[gk], mean[N + gk], mean[2 * N + gk]};
  const float ls[3] = {log_scale[gk], log_scale[N + gk], log_scale[2 * N + gk]};
  const float q[4] = {quat[gk], quat[N + gk], quat[2 * N + gk], quat[3 * N + gk]};
  const ProjF P = project_f(cam, m, ls, q, opl[gk]);
  int rr = 0;
  int2 rc;
  const bool nonempty = tile_rect_of(P, tab.gx[v], tab.gy[v], rc, rr);
  rect[r] = rc;
  const uint32_t kout = nonempty ? __float_as_uint(P.pz) : 0xFFFFFFFFu;
  key[r] = kout;
  if (rec && nonempty) {
    rec[3 * r + 0] = make_float4(P.ux, P.uy, P.pz, P.o);
    rec[3 * r + 1] = make_float4(gs_conic_scale_diag(P.k1), gs_conic_scale_off(P.k2), gs_conic_scale_diag(P.k3),
                                 mp[gk]);
    rec[3 * r + 2] = make_float4(color[gk], color[N + gk], color[2 * N + gk], 0.f);
  }
  if (mean2d) {
    mean2d[r] = P.ux;
    mean2d[M + r] = P.uy;
  }
  if (conic) {
    conic[r] = P.k1;
    conic[M + r] = P.k2;
    conic[2 * M + r] = P.k3;
  }
  if (depth) depth[r] = P.pz;
  if (opacity) opacity[r] = P.o;
  if (radius) radius[r] = P.kept ? rr : 0;
  return kout;
}

__global__ __launch_bounds__(PBLOCK) void project_kernel(ViewTab tab, const gs_camera* __restrict__ cams,
                                                         const float* __restrict__ mean,
                                                         const float* __restrict__ log_scale,
                                                         const float* __restrict__ quat,
                                                         const float* __restrict__ opl,
                                                         const float* __restrict__ color,
                                                         const float* __restrict__ mp, float4* __restrict__ rec,
                                                         int2* __restrict__ rect,
                                                         uint32_t* __restrict__ key, float* __restrict__ mean2d,
                                                         float* __restrict__ conic, float* __restrict__ depth,
                                                         float* __restrict__ opacity, int32_t* __restrict__ radius,
                                                         uint32_t* __restrict__ key_hist) {
  extern __shared__ uint32_t s_hist[];  // 4096 bins when key_hist is set
  const int v = blockIdx.y;
  const int64_t npad = tab.npad[v];
  const int64_t base = (int64_t)blockIdx.x * PBLOCK * PITEMS;
  if (base >= npad) return;  // uniform per workgroup
  if (key_hist) {
    for (int i = threadIdx.x; i < 4096; i += PBLOCK) s_hist[i] = 0;
    __syncthreads();
  }
  const gs_camera cam = cams[v];
#pragma unroll
  for (int it = 0; it < PITEMS; ++it) {
    const int64_t k = base + it * PBLOCK + threadIdx.x;
    if (k < npad) {
      const uint32_t kv =
          project_one(tab, cam, mean, log_scale, quat, opl, color, mp, rec, rect, key, mean2d, conic, depth,
                      opacity, radius, v, k);
      if (key_hist && kv != 0xFFFFFFFFu) atomicAdd(&s_hist[kv >> 20], 1u);
    }
  }
  if (key_hist) {
    __syncthreads();
    for (int i = threadIdx.x; i < 4096; i += PBLOCK) {
      const uint32_t c = s_hist[i];
      if (c) atomicAdd(&key_hist[(int64_t)v * 4096 + i], c);
    }
  }
}

// The prefix path's projection when no planar output is asked for: only the
// depth key of every Gaussian (from the cheap screen test, which never drops
// a Gaussian the exact projection keeps) and the key histogram. gs_bin_sort
// then projects the few selected Gaussians exactly, writes their rects and
// compositing records and drops those the exact test culls. Reads 28 bytes
// per Gaussian (mean, log-scale, opacity logit) and writes 4.
__global__ __launch_bounds__(PBLOCK) void project_key_kernel(ViewTab tab, const gs_camera* __restrict__ cams,
                                                             const float* __restrict__ mean,
                                                             const float* __restrict__ log_scale,
                                                             const float* __restrict__ opl, uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ key_hist) {
  __shared__ uint32_t s_hist[4096];
  const int v = blockIdx.y;
  const int64_t npad = tab.npad[v];
  const int64_t base = (int64_t)blockIdx.x * PBLOCK * PITEMS;
  if (base >= npad) return;  // uniform per workgroup
  for (int i = threadIdx.x; i < 4096; i += PBLOCK) s_hist[i] = 0;
  const gs_camera cam = cams[v];
  const int64_t N = tab.ng, nv = tab.n[v], goff = tab.g_off[v], roff = tab.r_off[v];
  const int gx = tab.gx[v], gy = tab.gy[v];
  // every load of the workgroup's records in flight before the first is used
  float m[PITEMS][3], ls[PITEMS][3], ol[PITEMS];
#pragma unroll
  for (int it = 0; it < PITEMS; ++it) {
    const int64_t k = base + it * PBLOCK + threadIdx.x;
    const int64_t gk = goff + (k < nv ? k : 0);
    m[it][0] = mean[gk];
    m[it][1] = mean[N + gk];
    m[it][2] = mean[2 * N + gk];
    ls[it][0] = log_scale[gk];
    ls[it][1] = log_scale[N + gk];
    ls[it][2] = log_scale[2 * N + gk];
    ol[it] = opl[gk];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < PITEMS; ++it) {
    const int64_t k = base + it * PBLOCK + threadIdx.x;
    if (k >= npad) continue;
    const uint32_t kv = k < nv ? screen_key(cam, m[it], ls[it], ol[it], gx, gy) : 0xFFFFFFFFu;
    key[roff + k] = kv;
    if (kv != 0xFFFFFFFFu) atomicAdd(&s_hist[kv >> 20], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4096; i += PBLOCK) {
    const uint32_t c = s_hist[i];
    if (c) atomicAdd(&key_hist[(int64_t)v * 4096 + i], c);
  }
}

}  // namespace

gs_status launch_project(gs_ctx* ctx, const ViewTab& tab, const gs_camera* cams, const gs_gaussians* g,
                         gs_proj* p, hipStream_t s) {
  int64_t maxn = 0;
  for (int v = 0; v < tab.nv; ++v) maxn = tab.npad[v] > maxn ? tab.npad[v] : maxn;
  if (maxn == 0) return GS_OK;
  dim3 grid((unsigned)((maxn + PBLOCK * PITEMS - 1) / (PBLOCK * PITEMS)), tab.nv);
  const bool planar = p->mean2d || p->conic || p->depth || p->opacity || p->radius;
  p->keys_only = p->key_hist && !planar && !ctx->exact_keys ? 1 : 0;
  if (p->keys_only) {
    GS_LAUNCH(ctx, project_key_kernel, grid, dim3(PBLOCK), 0, s, tab, cams, g->mean, g->log_scale, g->opacity_logit,
              p->depth_key, p->key_hist);
    return gs_check_launch(ctx, "project");
  }
  GS_LAUNCH(ctx, project_kernel, grid, dim3(PBLOCK), p->key_hist ? 4096 * 4 : 0, s, tab, cams, g->mean,
            g->log_scale, g->quat, g->opacity_logit, g->color, g->mp, p->key_hist ? nullptr : (float4*)p->rec,
            (int2*)p->rect, p->depth_key, p->mean2d, p->conic, p->depth, p->opacity, p->radius, p->key_hist);
  return gs_check_launch(ctx, "project");
}
