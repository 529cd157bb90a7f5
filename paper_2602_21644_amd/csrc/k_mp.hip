// gs_mp_update: one frame of the per-Gaussian motion-probability update.
//
//  1. region statistics of the residual cue over valid pixels (Eq. 4):
//     per-block float64 sums of (count, e, e^2) per region, reduced in a fixed
//     order (deterministic);
//  2. per pixel: MP_geo (Eq. 5 with the small-sigma rule), instance prior and
//     confidence (Eq. 2), gain (Eq. 7) and fused M_p (Eq. 6);
//  3. per Gaussian: valid pixels within radius_px of the projected mean
//     (Eq. 1, one scale; membership decided in float32 without fma), kernel-
//     weighted mean M_hat (Eq. 8), variance of M_p, std of e, uncertainty U
//     (Eq. 10); frame min/max of U by integer atomics on ordered bit patterns;
//  4. per Gaussian: normalised U, rate (Eq. 11), stale-prior factor (Eq. 17)
//     and the state update (Eq. 9, or the log-odds variant);
//  5. lower medians of M^t and U~ over observed Gaussians by an exact 4-pass
//     8-bit radix select on the float bit patterns (values are >= 0);
//  6. threshold tau = max(median, 0.5), labels (Eq. 12), prune flags, and the
//     frame uncertainty (Eq. 13).
#include "gs_internal.h"

namespace {

constexpr int MAXR = 16;         // regions: background + up to 15 instances
constexpr int PIX_ITEMS = 16;    // pixels per thread in the region pass
constexpr int REG_TILE = GS_BLOCK * PIX_ITEMS;

struct MpScal {
  uint32_t umin, umax;      // ordered-int encodings of min/max U
  uint32_t n_obs, n_dyn, n_prune, pad0;
  uint32_t prefix[2], rank[2];
  uint32_t hist[2][256];
  float region[MAXR][4];    // mu, sigma, e_ub, Gamma_geo
};

__device__ __forceinline__ uint32_t f2ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

__device__ __forceinline__ double block_sum_d(double x, double* s) {
  x = wave_sum_to_lane63_d(x);
  if (__lane_id() == 63) s[threadIdx.x >> 6] = x;
  __syncthreads();
  const double r = s[0] + s[1] + s[2] + s[3];
  __syncthreads();
  return r;
}

__device__ __forceinline__ float residual(const float* D, const float* Dg, const float* C, const float* Cg, int64_t P,
                                          int64_t i, float beta) {
  float e = fabsf(D[i] - Dg[i]);
  if (beta != 0.f) e += beta * (fabsf(C[i] - Cg[i]) + fabsf(C[P + i] - Cg[P + i]) + fabsf(C[2 * P + i] - Cg[2 * P + i]));
  return e;
}

__global__ __launch_bounds__(GS_BLOCK) void mp_region_kernel(int64_t npix, int64_t P, int K,
                                                             const float* __restrict__ D, const float* __restrict__ Dg,
                                                             const float* __restrict__ C,
                                                             const float* __restrict__ Cg,
                                                             const int32_t* __restrict__ inst, float beta,
                                                             float* __restrict__ e_out, double* __restrict__ part) {
  __shared__ double s[4];
  const int64_t base = (int64_t)blockIdx.x * REG_TILE;
  float ev[PIX_ITEMS];
  int rv[PIX_ITEMS];
#pragma unroll
  for (int i = 0; i < PIX_ITEMS; ++i) {
    const int64_t p = base + i * GS_BLOCK + threadIdx.x;
    rv[i] = -1;
    ev[i] = 0.f;
    if (p < npix) {
      const float e = residual(D, Dg, C, Cg, P, p, beta);
      e_out[p] = e;
      if (Dg[p] > 0.f) {
        ev[i] = e;
        rv[i] = min(max(inst[p], 0), K);
      }
    }
  }
  for (int r = 0; r <= K; ++r) {
    double c = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int i = 0; i < PIX_ITEMS; ++i)
      if (rv[i] == r) {
        c += 1.0;
        s1 += (double)ev[i];
        s2 += (double)ev[i] * (double)ev[i];
      }
    c = block_sum_d(c, s);
    s1 = block_sum_d(s1, s);
    s2 = block_sum_d(s2, s);
    if (threadIdx.x == 0) {
      double* o = part + ((int64_t)blockIdx.x * MAXR + r) * 3;
      o[0] = c;
      o[1] = s1;
      o[2] = s2;
    }
  }
}

__global__ void mp_region_final_kernel(const double* __restrict__ part, int nb, int K, float lambda_e, float e_floor,
                                       float sigma_g, MpScal* __restrict__ sc) {
  const int r = threadIdx.x;
  if (threadIdx.x == 0) {
    sc->umin = 0xFFFFFFFFu;
    sc->umax = 0u;
    sc->n_obs = sc->n_dyn = sc->n_prune = 0;
  }
  if (r > K) return;
  double c = 0, s1 = 0, s2 = 0;
  for (int b = 0; b < nb; ++b) {
    const double* o = part + ((int64_t)b * MAXR + r) * 3;
    c += o[0];
    s1 += o[1];
    s2 += o[2];
  }
  double mu = 0, sd = 0;
  if (c > 0) {
    mu = s1 / c;
    sd = sqrt(fmax(s2 / c - mu * mu, 0.0));
  }
  const double ub = fmax(mu + (double)lambda_e * sd, (double)e_floor);
  sc->region[r][0] = (float)mu;
  sc->region[r][1] = (float)sd;
  sc->region[r][2] = (float)ub;
  sc->region[r][3] = (float)exp(-sd / (double)sigma_g);
}

__global__ __launch_bounds__(GS_BLOCK) void mp_pixel_kernel(int64_t npix, int K, const float* __restrict__ e_in,
                                                            const int32_t* __restrict__ inst,
                                                            const float* __restrict__ prior,
                                                            const float* __restrict__ conf,
                                                            const float* __restrict__ mlp, float sigma_small,
                                                            const MpScal* __restrict__ sc, float* __restrict__ Mp,
                                                            float* __restrict__ e_copy) {
  const int64_t p = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  if (p >= npix) return;
  const int r = min(max(inst[p], 0), K);
  const float e = e_in[p];
  if (e_copy) e_copy[p] = e;
  if (mlp) {
    Mp[p] = mlp[p];
    return;
  }
  const float mu = sc->region[r][0], sd = sc->region[r][1], ub = sc->region[r][2], gg = sc->region[r][3];
  const float et = sd < sigma_small ? mu : e;
  const float geo = ub > 0.f ? fminf(fmaxf(et / ub, 0.f), 1.f) : 0.f;
  const float gi = conf[r];
  const float den = gi + gg;
  const float Kp = den > 0.f ? gg / den : 0.5f;
  Mp[p] = (1.f - Kp) * prior[r] + Kp * geo;
}

struct GaussOut {
  float* Mhat;
  float* sde;
  float* U;
  uint8_t* obs;
};

__global__ __launch_bounds__(GS_BLOCK) void mp_gauss_kernel(ViewTab tab, const float* __restrict__ mean2d,
                                                            const uint32_t* __restrict__ key,
                                                            const float* __restrict__ Dg,
                                                            const float* __restrict__ Mp,
                                                            const float* __restrict__ e_in,
                                                            const float* __restrict__ mp, float radius, float sigma_w,
                                                            float lambda_u, float eps, GaussOut go,
                                                            MpScal* __restrict__ sc) {
  __shared__ uint32_t s_min, s_max, s_cnt;
  if (threadIdx.x == 0) {
    s_min = 0xFFFFFFFFu;
    s_max = 0u;
    s_cnt = 0u;
  }
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  const int W = tab.W[0], H = tab.H[0];
  const int64_t M = tab.nrec;
  if (k < tab.n[0]) {
    const int64_t r = tab.r_off[0] + k;
    bool obs = false;
    float Mhat = 0.f, sde = 0.f, U = 0.f;
    const float ux = mean2d[r], uy = mean2d[M + r];
    const bool vis = key[r] != 0xFFFFFFFFu && ux >= 0.f && ux <= (float)(W - 1) && uy >= 0.f && uy <= (float)(H - 1);
    if (vis) {
      const float r2 = __fmul_rn(radius, radius);
      const int rr = (int)ceilf(radius) + 1;
      const int cx = (int)floorf(ux), cy = (int)floorf(uy);
      const int x0 = max(0, cx - rr), x1 = min(W - 1, cx + rr);
      const int y0 = max(0, cy - rr), y1 = min(H - 1, cy + rr);
      const float inv2 = 1.0f / (2.0f * sigma_w * sigma_w);
      int n = 0;
      float sw = 0.f, swm = 0.f, sm = 0.f, se = 0.f;
      for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
          const float dx = __fsub_rn((float)x, ux), dy = __fsub_rn((float)y, uy);
          const float d2 = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
          const int64_t p = (int64_t)y * W + x;
          if (d2 <= r2 && Dg[p] > 0.f) {
            const float w = __expf(-d2 * inv2);
            const float m = Mp[p];
            ++n;
            sw += w;
            swm += w * m;
            sm += m;
            se += e_in[p];
          }
        }
      if (n > 0) {
        obs = true;
        const float mm = sm / n, me = se / n;
        float vm = 0.f, ve = 0.f;
        for (int y = y0; y <= y1; ++y)
          for (int x = x0; x <= x1; ++x) {
            const float dx = __fsub_rn((float)x, ux), dy = __fsub_rn((float)y, uy);
            const float d2 = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
            const int64_t p = (int64_t)y * W + x;
            if (d2 <= r2 && Dg[p] > 0.f) {
              const float a = Mp[p] - mm, b = e_in[p] - me;
              vm += a * a;
              ve += b * b;
            }
          }
        const float var = vm / n;
        sde = sqrtf(ve / n);
        Mhat = swm / sw;
        const float M0 = mp[tab.g_off[0] + k];
        U = -M0 * logf(M0 + eps) - (1.f - M0) * logf(1.f - M0 + eps) + lambda_u * var;
        atomicMin(&s_min, f2ord(U));
        atomicMax(&s_max, f2ord(U));
        atomicAdd(&s_cnt, 1u);
      }
    }
    go.Mhat[k] = Mhat;
    go.sde[k] = sde;
    go.U[k] = U;
    go.obs[k] = obs ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_cnt > 0) {
    atomicMin(&sc->umin, s_min);
    atomicMax(&sc->umax, s_max);
    atomicAdd(&sc->n_obs, s_cnt);
  }
}

__global__ __launch_bounds__(GS_BLOCK) void mp_state_kernel(ViewTab tab, GaussOut go, const MpScal* __restrict__ sc,
                                                            float sigma_c, float lambda_u, float amin, float amax,
                                                            float rho, int seg, int mode, int u_norm, float le,
                                                            float lmax, float* __restrict__ mp,
                                                            float* __restrict__ Ut_out, float* __restrict__ a_out) {
  const int64_t k = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  if (k >= tab.n[0]) return;
  const int64_t gk = tab.g_off[0] + k;
  if (!go.obs[k]) {
    Ut_out[gk] = 0.f;
    a_out[gk] = 0.f;
    return;
  }
  const float U = go.U[k];
  float Ut;
  if (u_norm == 0) {
    const float umin = ord2f(sc->umin), umax = ord2f(sc->umax);
    Ut = umax > umin ? (U - umin) / (umax - umin) : 0.f;
  } else {
    Ut = fminf(fmaxf(U / (0.69314718055994531f + 0.25f * lambda_u), 0.f), 1.f);
  }
  const float Cg = __expf(-go.sde[k] / sigma_c);
  float a = amin + (amax - amin) * (1.f - Ut) * Cg;
  a = fminf(fmaxf(a, amin), amax);
  if (!seg) a *= rho;
  const float m0 = mp[gk], mh = go.Mhat[k];
  float m1;
  if (mode == 0) {
    m1 = (1.f - a) * m0 + a * mh;
  } else {
    const float p0 = fminf(fmaxf(m0, le), 1.f - le), p1 = fminf(fmaxf(mh, le), 1.f - le);
    const float l = fminf(fmaxf(logf(p0 / (1.f - p0)) + a * logf(p1 / (1.f - p1)), -lmax), lmax);
    m1 = 1.f / (1.f + expf(-l));
  }
  mp[gk] = m1;
  Ut_out[gk] = Ut;
  a_out[gk] = a;
}

// Radix select: pass `pass` (0 = bits 31..24) histograms the digit of every
// observed value whose higher digits match the running prefix.
__global__ __launch_bounds__(GS_BLOCK) void mp_sel_hist_kernel(int64_t n, int64_t g_off, const uint8_t* __restrict__ obs,
                                                               const float* __restrict__ v0,
                                                               const float* __restrict__ v1, int pass,
                                                               MpScal* __restrict__ sc) {
  __shared__ uint32_t h[2][256];
  h[0][threadIdx.x] = 0;
  h[1][threadIdx.x] = 0;
  __syncthreads();
  const int shift = 24 - 8 * pass;
  const uint32_t hmask = pass == 0 ? 0u : (0xFFFFFFFFu << (shift + 8));
  const uint32_t p0 = sc->prefix[0], p1 = sc->prefix[1];
  for (int64_t k = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x; k < n; k += (int64_t)gridDim.x * GS_BLOCK) {
    if (!obs[k]) continue;
    const uint32_t a = __float_as_uint(v0[g_off + k]);
    const uint32_t b = __float_as_uint(v1[g_off + k]);
    if ((a & hmask) == (p0 & hmask)) atomicAdd(&h[0][(a >> shift) & 255u], 1u);
    if ((b & hmask) == (p1 & hmask)) atomicAdd(&h[1][(b >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[0][threadIdx.x]) atomicAdd(&sc->hist[0][threadIdx.x], h[0][threadIdx.x]);
  if (h[1][threadIdx.x]) atomicAdd(&sc->hist[1][threadIdx.x], h[1][threadIdx.x]);
}

__global__ void mp_sel_pick_kernel(int pass, MpScal* __restrict__ sc) {
  const int which = threadIdx.x;  // 2 threads
  if (which < 2) {
    if (pass == 0) {
      sc->rank[which] = sc->n_obs > 0 ? (sc->n_obs - 1) / 2 : 0;
      sc->prefix[which] = 0;
    }
    const int shift = 24 - 8 * pass;
    uint32_t rank = sc->rank[which], acc = 0;
    int d = 0;
    for (; d < 256; ++d) {
      const uint32_t c = sc->hist[which][d];
      if (rank < acc + c) break;
      acc += c;
    }
    if (d > 255) d = 255;
    sc->rank[which] = rank - acc;
    sc->prefix[which] |= (uint32_t)d << shift;
    for (int i = 0; i < 256; ++i) sc->hist[which][i] = 0;
  }
}

__global__ void mp_sel_reset_kernel(MpScal* __restrict__ sc) {
  for (int i = threadIdx.x; i < 512; i += blockDim.x) (&sc->hist[0][0])[i] = 0;
  if (threadIdx.x < 2) {
    sc->prefix[threadIdx.x] = 0;
    sc->rank[threadIdx.x] = 0;
  }
}

__global__ __launch_bounds__(GS_BLOCK) void mp_label_kernel(ViewTab tab, const float* __restrict__ mp,
                                                            float prune_above, MpScal* __restrict__ sc,
                                                            uint8_t* __restrict__ dyn, uint8_t* __restrict__ prune) {
  __shared__ uint32_t s_d, s_p;
  if (threadIdx.x == 0) {
    s_d = 0;
    s_p = 0;
  }
  __syncthreads();
  const float med = sc->n_obs > 0 ? __uint_as_float(sc->prefix[0]) : 0.f;
  const float tau = sc->n_obs > 0 ? fmaxf(med, 0.5f) : 0.5f;
  const int64_t k = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  if (k < tab.n[0]) {
    const int64_t gk = tab.g_off[0] + k;
    const float m = mp[gk];
    const bool d = m > tau, p = m > prune_above;
    dyn[gk] = d;
    prune[gk] = p;
    if (d) atomicAdd(&s_d, 1u);
    if (p) atomicAdd(&s_p, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_d) atomicAdd(&sc->n_dyn, s_d);
    if (s_p) atomicAdd(&sc->n_prune, s_p);
  }
}

__global__ void mp_stats_kernel(const MpScal* __restrict__ sc, float* __restrict__ stats) {
  if (threadIdx.x != 0) return;
  const bool any = sc->n_obs > 0;
  const float med = any ? __uint_as_float(sc->prefix[0]) : 0.f;
  stats[0] = any ? __uint_as_float(sc->prefix[1]) : 0.f;
  stats[1] = any ? fmaxf(med, 0.5f) : 0.5f;
  stats[2] = (float)sc->n_obs;
  stats[3] = (float)sc->n_dyn;
  stats[4] = (float)sc->n_prune;
  stats[5] = any ? ord2f(sc->umin) : 0.f;
  stats[6] = any ? ord2f(sc->umax) : 0.f;
  stats[7] = med;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct MpWs {
  size_t e, Mp, part, scal, Mhat, sde, U, obs, bytes;
};

MpWs mp_layout(int64_t n, int64_t P) {
  MpWs L;
  size_t o = 0;
  const int64_t nb = (P + REG_TILE - 1) / REG_TILE;
  L.e = o; o += al(P * 4);
  L.Mp = o; o += al(P * 4);
  L.part = o; o += al((size_t)(nb > 0 ? nb : 1) * MAXR * 3 * 8);
  L.scal = o; o += al(sizeof(MpScal));
  L.Mhat = o; o += al(n * 4);
  L.sde = o; o += al(n * 4);
  L.U = o; o += al(n * 4);
  L.obs = o; o += al(n);
  L.bytes = o;
  return L;
}

}  // namespace

size_t mp_ws_bytes(const ViewTab& tab, int64_t npix) { return mp_layout(tab.n[0], npix).bytes; }

gs_status launch_mp_update(gs_ctx* ctx, const ViewTab& tab, const gs_proj* proj, const gs_image* img,
                           const gs_target* tgt, const gs_mp_frame* fr, const gs_mp_params* pp, float* mp,
                           gs_mp_out* out, char* ws, hipStream_t s) {
  const int64_t P = tab.npix, n = tab.n[0];
  const MpWs L = mp_layout(n, P);
  float* e = (float*)(ws + L.e);
  float* Mp = out->M_p ? out->M_p : (float*)(ws + L.Mp);
  double* part = (double*)(ws + L.part);
  MpScal* sc = (MpScal*)(ws + L.scal);
  GaussOut go{(float*)(ws + L.Mhat), (float*)(ws + L.sde), (float*)(ws + L.U), (uint8_t*)(ws + L.obs)};
  const int K = fr->n_inst;
  const int nb = (int)((P + REG_TILE - 1) / REG_TILE);
  if (nb > 0)
    GS_LAUNCH(ctx, mp_region_kernel, dim3(nb), dim3(GS_BLOCK), 0, s, P, P, K, img->depth, tgt->depth, img->color,
                       tgt->color, fr->instance_id, pp->beta_color, e, part);
  GS_LAUNCH(ctx, mp_region_final_kernel, dim3(1), dim3(64), 0, s, part, nb, K, pp->lambda_e, pp->e_floor,
                     pp->sigma_g, sc);
  if (P > 0)
    GS_LAUNCH(ctx, mp_pixel_kernel, dim3((unsigned)((P + GS_BLOCK - 1) / GS_BLOCK)), dim3(GS_BLOCK), 0, s, P, K,
                       e, fr->instance_id, fr->inst_prior, fr->inst_conf, fr->mlp_mp, pp->sigma_small, sc, Mp,
                       out->e);
  const unsigned gb = (unsigned)((n + GS_BLOCK - 1) / GS_BLOCK);
  if (n > 0) {
    GS_LAUNCH(ctx, mp_gauss_kernel, dim3(gb), dim3(GS_BLOCK), 0, s, tab, proj->mean2d, proj->depth_key,
                       tgt->depth, Mp, e, mp, pp->radius_px, pp->sigma_w, pp->lambda_u, pp->eps, go, sc);
    GS_LAUNCH(ctx, mp_state_kernel, dim3(gb), dim3(GS_BLOCK), 0, s, tab, go, sc, pp->sigma_c, pp->lambda_u,
                       pp->alpha_min, pp->alpha_max, pp->rho, fr->seg_updated, pp->mode, pp->u_norm, pp->logodds_eps,
                       pp->logodds_max, mp, out->U_tilde, out->alpha);
  }
  GS_LAUNCH(ctx, mp_sel_reset_kernel, dim3(1), dim3(GS_BLOCK), 0, s, sc);
  const unsigned sb = gb < 1024 ? (gb > 0 ? gb : 1) : 1024;
  for (int pass = 0; pass < 4; ++pass) {
    GS_LAUNCH(ctx, mp_sel_hist_kernel, dim3(sb), dim3(GS_BLOCK), 0, s, n, tab.g_off[0], go.obs, mp, out->U_tilde,
                       pass, sc);
    GS_LAUNCH(ctx, mp_sel_pick_kernel, dim3(1), dim3(64), 0, s, pass, sc);
  }
  if (n > 0)
    GS_LAUNCH(ctx, mp_label_kernel, dim3(gb), dim3(GS_BLOCK), 0, s, tab, mp, pp->prune_above, sc, out->dynamic,
                       out->prune);
  GS_LAUNCH(ctx, mp_stats_kernel, dim3(1), dim3(64), 0, s, sc, out->stats);
  return gs_check_launch(ctx, "mp_update");
}
