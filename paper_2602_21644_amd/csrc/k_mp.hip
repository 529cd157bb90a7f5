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
//  5. lower medians of M^t and U~ over observed Gaussians by an exact 3-pass
//     radix select (digits of 11, 11 and 10 bits) on the float bit patterns
//     (values are >= 0);
//  6. threshold tau = max(median, 0.5), labels (Eq. 12), prune flags, and the
//     frame uncertainty (Eq. 13).
#include "gs_internal.h"

namespace {

constexpr int MAXR = 16;         // regions: background + up to 15 instances
constexpr int PIX_ITEMS = 4;     // pixels per thread in the region pass
constexpr int REG_TILE = GS_BLOCK * PIX_ITEMS;
constexpr int SEL_BLOCKS = 256;
constexpr int SEL_COPIES = 8;  // histogram copies, one per XCD
constexpr int SEL_PASSES = 3;
constexpr int SEL_BINS = 2048;  // bins per value and pass (the last pass uses 1024)
constexpr int SEL_HIST = 2 * SEL_BINS;  // both values' bins in one copy
// digit of pass p: bits [sel_shift(p), sel_shift(p) + sel_width(p))
__device__ __forceinline__ int sel_shift(int pass) { return pass == 0 ? 21 : pass == 1 ? 10 : 0; }
__device__ __forceinline__ int sel_width(int pass) { return pass == 2 ? 10 : 11; }

struct MpScal {
  uint32_t umin, umax;      // ordered-int encodings of min/max U
  uint32_t n_obs, n_dyn, n_prune, pad0;
  uint32_t prefix[2], rank[2];
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
  x = wave_sum_all_d(x);
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
                                                             float* __restrict__ e_out, double* __restrict__ part,
                                                             int64_t nrows) {
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
  // per-wave partial sums of every region (no block barrier), stored
  // [region][count, sum e, sum e^2][row] so that the final pass reads each
  // region's rows contiguously
  const int64_t row = (int64_t)blockIdx.x * (GS_BLOCK / 64) + (threadIdx.x >> 6);
  for (int r = 0; r <= K; ++r) {
    double c = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int i = 0; i < PIX_ITEMS; ++i)
      if (rv[i] == r) {
        c += 1.0;
        s1 += (double)ev[i];
        s2 += (double)ev[i] * (double)ev[i];
      }
    c = wave_sum_all_d(c);
    s1 = wave_sum_all_d(s1);
    s2 = wave_sum_all_d(s2);
    if (__lane_id() == 0) {
      double* o = part + (int64_t)r * 3 * nrows + row;
      o[0] = c;
      o[nrows] = s1;
      o[2 * nrows] = s2;
    }
  }
}

// One wave per region sums the per-wave partials (rows) in a fixed order.
__global__ __launch_bounds__(MAXR * 64) void mp_region_final_kernel(const double* __restrict__ part, int nrows, int K,
                                                                    float lambda_e, float e_floor, float sigma_g,
                                                                    MpScal* __restrict__ sc, float* __restrict__ judge) {
  const int r = threadIdx.x >> 6, lane = __lane_id();
  if (judge && threadIdx.x == 0) {  // the surrogate judge accumulates in the pixel pass that follows
    judge[0] = 0.f;
    judge[1] = 0.f;
  }
  if (r > K) return;
  double c = 0, s1 = 0, s2 = 0;
  // each lane has kRowUnroll rows' loads in flight before it adds them, in
  // row order
  constexpr int kRowUnroll = 8;
  for (int b0 = lane; b0 < nrows; b0 += kRowUnroll * 64) {
    double x[kRowUnroll][3];
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u) {
      const int b = b0 + u * 64;
      const double* o = part + (int64_t)r * 3 * nrows + b;
#pragma unroll
      for (int q = 0; q < 3; ++q) x[u][q] = b < nrows ? o[(int64_t)q * nrows] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u) {
      c += x[u][0];
      s1 += x[u][1];
      s2 += x[u][2];
    }
  }
  c = wave_sum_all_d(c);
  s1 = wave_sum_all_d(s1);
  s2 = wave_sum_all_d(s2);
  if (lane != 0) return;
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
                                                            float* __restrict__ e_copy, const float* __restrict__ Dg,
                                                            float2* __restrict__ pk, float* __restrict__ judge) {
  const int64_t p = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  const bool live = p < npix;
  float dev = 0.f, cnt = 0.f;
  if (live) {
    const int r = min(max(inst[p], 0), K);
    const float e = e_in[p];
    if (e_copy) e_copy[p] = e;
    const float mu = sc->region[r][0], sd = sc->region[r][1], ub = sc->region[r][2], gg = sc->region[r][3];
    const float et = sd < sigma_small ? mu : e;
    const float geo = ub > 0.f ? fminf(fmaxf(et / ub, 0.f), 1.f) : 0.f;
    const float gi = conf[r];
    const float den = gi + gg;
    const float Kp = den > 0.f ? gg / den : 0.5f;
    const float plain = (1.f - Kp) * prior[r] + Kp * geo;
    const bool seen = Dg[p] > 0.f;
    float m = plain;
    if (mlp) {
      m = mlp[p];
      if (seen) {
        dev = fabsf(m - plain);
        cnt = 1.f;
      }
    }
    Mp[p] = m;
    // (M_p, e) packed for the per-Gaussian windows, e = -1 where no depth was
    // observed (e >= 0 elsewhere): 8 bytes per pixel, so a frame's pixels
    // stay in one XCD's L2
    pk[p] = make_float2(m, seen ? e : -1.f);
  }
  if (judge && mlp) {  // uniform: one atomic pair per wave
    dev = wave_sum_to_lane63(dev);
    cnt = wave_sum_to_lane63(cnt);
    if (__lane_id() == 63 && cnt > 0.f) {
      atomicAdd(&judge[0], dev);
      atomicAdd(&judge[1], cnt);
    }
  }
}

struct GaussOut {
  float* Mhat;
  float* sde;
  float* U;
  uint8_t* obs;
};

__global__ __launch_bounds__(GS_BLOCK) void mp_gauss_kernel(ViewTab tab, const float* __restrict__ mean2d,
                                                            const uint32_t* __restrict__ key,
                                                            const float2* __restrict__ pk,
                                                            const float* __restrict__ mp, float radius, float sigma_w,
                                                            float lambda_u, float eps, GaussOut go,
                                                            uint32_t* __restrict__ part_u) {
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
  uint32_t umin = 0xFFFFFFFFu, umax = 0u;  // order-preserving bits of U when observed
  bool seen = false;
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
      // one pass over the window: weighted mean of M_p, and the population
      // variances of M_p and e from sums shifted by the first valid sample
      // (exact zero for constant samples)
      int n = 0;
      float sw = 0.f, swm = 0.f, km = 0.f, ke = 0.f, am = 0.f, am2 = 0.f, ae = 0.f, ae2 = 0.f;
      auto take = [&](const float2& v, float d2) {
        const float w = __expf(-d2 * inv2);
        if (n == 0) {
          km = v.x;
          ke = v.y;
        }
        ++n;
        sw += w;
        swm += w * v.x;
        const float a = v.x - km, b = v.y - ke;
        am += a;
        am2 += a * a;
        ae += b;
        ae2 += b * b;
      };
      if (radius <= 2.0f) {
        // every pixel within 2 px lies in the 5x5 box from (ceil(ux-2),
        // ceil(uy-2)); its loads are issued together, visited in the same
        // row-major order as the general loop below
        const int xs = (int)ceilf(ux - 2.0f), ys = (int)ceilf(uy - 2.0f);
        float2 v[25];
        float dd[25];
        bool in[25];
#pragma unroll
        for (int i = 0; i < 25; ++i) {
          const int x = xs + i % 5, y = ys + i / 5;
          const float dx = __fsub_rn((float)x, ux), dy = __fsub_rn((float)y, uy);
          dd[i] = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
          in[i] = x >= x0 && x <= x1 && y >= y0 && y <= y1 && dd[i] <= r2;
          v[i] = in[i] ? pk[(int64_t)y * W + x] : make_float2(0.f, -1.f);
        }
#pragma unroll
        for (int i = 0; i < 25; ++i)
          if (in[i] && v[i].y >= 0.f) take(v[i], dd[i]);
      } else {
        for (int y = y0; y <= y1; ++y)
          for (int x = x0; x <= x1; ++x) {
            const float dx = __fsub_rn((float)x, ux), dy = __fsub_rn((float)y, uy);
            const float d2 = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
            if (d2 <= r2) {
              const float2 v = pk[(int64_t)y * W + x];
              if (v.y >= 0.f) take(v, d2);
            }
          }
      }
      if (n > 0) {
        obs = true;
        const float fn = (float)n;
        const float var = fmaxf(0.f, (am2 - am * am / fn) / fn);
        sde = sqrtf(fmaxf(0.f, (ae2 - ae * ae / fn) / fn));
        Mhat = swm / sw;
        const float M0 = mp[tab.g_off[0] + k];
        U = -M0 * logf(M0 + eps) - (1.f - M0) * logf(1.f - M0 + eps) + lambda_u * var;
      }
    }
    go.Mhat[k] = Mhat;
    go.sde[k] = sde;
    go.U[k] = U;
    go.obs[k] = obs ? 1 : 0;
    if (obs) {
      umin = f2ord(U);
      umax = umin;
      seen = true;
    }
  }
  // range and count of U over the block: per wave by shuffles, then one LDS
  // atomic per wave
  const uint32_t cnt = (uint32_t)__popcll(__ballot(seen));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    umin = min(umin, (uint32_t)__shfl_xor((int)umin, o, 64));
    umax = max(umax, (uint32_t)__shfl_xor((int)umax, o, 64));
  }
  if (__lane_id() == 0 && cnt) {
    atomicMin(&s_min, umin);
    atomicMax(&s_max, umax);
    atomicAdd(&s_cnt, cnt);
  }
  __syncthreads();
  // the block's partial (min, max, count), summed by mp_ureduce_kernel
  if (threadIdx.x == 0) {
    part_u[3 * (int64_t)blockIdx.x + 0] = s_min;
    part_u[3 * (int64_t)blockIdx.x + 1] = s_max;
    part_u[3 * (int64_t)blockIdx.x + 2] = s_cnt;
  }
}

// Range and count of U over all blocks of mp_gauss_kernel (one workgroup).
__global__ __launch_bounds__(1024) void mp_ureduce_kernel(const uint32_t* __restrict__ part_u, int nb,
                                                          MpScal* __restrict__ sc, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_v[3][16];
  // the selection's histogram copies start every update cleared
  for (int i = threadIdx.x; i < SEL_COPIES * SEL_HIST; i += 1024) hist[i] = 0;
  uint32_t mn = 0xFFFFFFFFu, mx = 0u, cnt = 0u;
  for (int b = threadIdx.x; b < nb; b += 1024) {
    mn = min(mn, part_u[3 * b + 0]);
    mx = max(mx, part_u[3 * b + 1]);
    cnt += part_u[3 * b + 2];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, o, 64));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    s_v[0][w] = mn;
    s_v[1][w] = mx;
    s_v[2][w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 16; ++i) {
      mn = min(mn, s_v[0][i]);
      mx = max(mx, s_v[1][i]);
    }
    uint32_t c = 0;
    for (int i = 0; i < 16; ++i) c += s_v[2][i];
    mn = min(mn, s_v[0][0]);
    mx = max(mx, s_v[1][0]);
    sc->umin = mn;
    sc->umax = mx;
    sc->n_obs = c;
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


// Radix select: pass `pass` histograms the digit (bits 31..21, 20..10, 9..0)
// of every observed value whose higher digits match the running prefix.
__global__ __launch_bounds__(GS_BLOCK) void mp_sel_hist_kernel(int64_t n, int64_t g_off, const uint8_t* __restrict__ obs,
                                                               const float* __restrict__ v0,
                                                               const float* __restrict__ v1, int pass,
                                                               const MpScal* __restrict__ sc,
                                                               uint32_t* __restrict__ part_h) {
  __shared__ uint32_t h[2][SEL_BINS];
  for (int i = threadIdx.x; i < SEL_BINS; i += GS_BLOCK) {
    h[0][i] = 0;
    h[1][i] = 0;
  }
  __syncthreads();
  const int shift = sel_shift(pass);
  const uint32_t dmask = (1u << sel_width(pass)) - 1u;
  const uint32_t hmask = pass == 0 ? 0u : (0xFFFFFFFFu << (shift + sel_width(pass)));
  const uint32_t p0 = pass == 0 ? 0u : sc->prefix[0], p1 = pass == 0 ? 0u : sc->prefix[1];
  for (int64_t base = (int64_t)blockIdx.x * GS_BLOCK; base < n; base += (int64_t)gridDim.x * GS_BLOCK) {
    const int64_t k = base + threadIdx.x;
    const bool o = k < n && obs[k];
    const uint32_t a = o ? __float_as_uint(v0[g_off + k]) : 0u;
    const uint32_t b = o ? __float_as_uint(v1[g_off + k]) : 0u;
    if (o && (a & hmask) == (p0 & hmask)) atomicAdd(&h[0][(a >> shift) & dmask], 1u);
    if (o && (b & hmask) == (p1 & hmask)) atomicAdd(&h[1][(b >> shift) & dmask], 1u);
  }
  __syncthreads();
  // added into the histogram copy of the XCD the workgroup runs on, so the
  // workgroups of different XCDs do not contend for one address; the pick
  // sums the copies and clears them
  uint32_t* hc = part_h + (__builtin_amdgcn_s_getreg((31 << 11) | 20) & (SEL_COPIES - 1)) * SEL_HIST;
  for (int i = threadIdx.x; i < SEL_BINS; i += GS_BLOCK) {
    if (h[0][i]) atomicAdd(&hc[i], h[0][i]);
    if (h[1][i]) atomicAdd(&hc[SEL_BINS + i], h[1][i]);
  }
}

// Sums the histogram copies (and clears them) and picks the digit holding
// the running rank (one workgroup: 512 threads per value, 4 bins each).
__global__ __launch_bounds__(1024) void mp_sel_pick_kernel(int pass, uint32_t* __restrict__ part_h,
                                                           MpScal* __restrict__ sc) {
  __shared__ uint32_t s_wsum[16];
  __shared__ uint32_t s_rank[2], s_prefix[2];
  const int t = threadIdx.x;
  if (t < 2) {  // the running state, read before any thread updates it
    s_rank[t] = pass == 0 ? (sc->n_obs > 0 ? (sc->n_obs - 1) / 2 : 0) : sc->rank[t];
    s_prefix[t] = pass == 0 ? 0u : sc->prefix[t];
  }
  const int which = t >> 9, d0 = 4 * (t & 511);  // value, first of this thread's bins
  uint32_t c4[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = which * SEL_BINS + d0 + q;
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < SEL_COPIES; ++c) {
      acc += part_h[c * SEL_HIST + i];
      part_h[c * SEL_HIST + i] = 0;
    }
    c4[q] = acc;
  }
  // inclusive scan of each value's bins: this thread's four, then over the
  // value's eight waves
  const uint32_t own = c4[0] + c4[1] + c4[2] + c4[3];
  const int lane = __lane_id(), w = t >> 6;
  uint32_t incl = own;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_wsum[w] = incl;
  __syncthreads();
  for (int i = which * 8; i < w; ++i) incl += s_wsum[i];
  uint32_t excl = incl - own;
  const uint32_t rank = s_rank[which], prefix = s_prefix[which];
  const int shift = sel_shift(pass), nbins = 1 << sel_width(pass);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int d = d0 + q;
    const uint32_t e1 = excl + c4[q];
    // the bin holding the rank; past every bin, the last one with all counted
    const bool hit = d < nbins && rank >= excl && rank < e1;
    const bool last = d == nbins - 1 && rank >= e1;
    if (hit || last) {
      sc->rank[which] = rank - (hit ? excl : e1);
      sc->prefix[which] = prefix | ((uint32_t)d << shift);
    }
    excl = e1;
  }
}

__global__ __launch_bounds__(GS_BLOCK) void mp_label_kernel(ViewTab tab, const float* __restrict__ mp,
                                                            float prune_above, const MpScal* __restrict__ sc,
                                                            uint8_t* __restrict__ dyn, uint8_t* __restrict__ prune,
                                                            uint32_t* __restrict__ part_l) {
  __shared__ uint32_t s_d, s_p;
  if (threadIdx.x == 0) {
    s_d = 0;
    s_p = 0;
  }
  __syncthreads();
  const float med = sc->n_obs > 0 ? __uint_as_float(sc->prefix[0]) : 0.f;
  const float tau = sc->n_obs > 0 ? fmaxf(med, 0.5f) : 0.5f;
  const int64_t k = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  bool d = false, p = false;
  if (k < tab.n[0]) {
    const int64_t gk = tab.g_off[0] + k;
    const float m = mp[gk];
    d = m > tau;
    p = m > prune_above;
    dyn[gk] = d;
    prune[gk] = p;
  }
  // counts per wave by ballot, one LDS atomic per wave
  const uint32_t cd = (uint32_t)__popcll(__ballot(d)), cp = (uint32_t)__popcll(__ballot(p));
  if (__lane_id() == 0) {
    if (cd) atomicAdd(&s_d, cd);
    if (cp) atomicAdd(&s_p, cp);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part_l[2 * (int64_t)blockIdx.x + 0] = s_d;
    part_l[2 * (int64_t)blockIdx.x + 1] = s_p;
  }
}

__global__ __launch_bounds__(1024) void mp_stats_kernel(MpScal* __restrict__ sc, const uint32_t* __restrict__ part_l,
                                                        int nb, float* __restrict__ stats) {
  __shared__ uint32_t s_v[2][16];
  uint32_t cd = 0, cp = 0;
  for (int b = threadIdx.x; b < nb; b += 1024) {
    cd += part_l[2 * b + 0];
    cp += part_l[2 * b + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cd += (uint32_t)__shfl_xor((int)cd, o, 64);
    cp += (uint32_t)__shfl_xor((int)cp, o, 64);
  }
  if (__lane_id() == 0) {
    s_v[0][threadIdx.x >> 6] = cd;
    s_v[1][threadIdx.x >> 6] = cp;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  cd = cp = 0;
  for (int i = 0; i < 16; ++i) {
    cd += s_v[0][i];
    cp += s_v[1][i];
  }
  sc->n_dyn = cd;
  sc->n_prune = cp;
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
  size_t e, Mp, pk, part, part_u, part_l, part_h, scal, Mhat, sde, U, obs, bytes;
};

MpWs mp_layout(int64_t n, int64_t P) {
  MpWs L;
  size_t o = 0;
  const int64_t nb = (P + REG_TILE - 1) / REG_TILE;
  const int64_t gb = (n + GS_BLOCK - 1) / GS_BLOCK;
  L.e = o; o += al(P * 4);
  L.Mp = o; o += al(P * 4);
  L.pk = o; o += al(P * 8);
  L.part = o; o += al((size_t)(nb > 0 ? nb : 1) * (GS_BLOCK / 64) * MAXR * 3 * 8);
  L.part_u = o; o += al((size_t)(gb > 0 ? gb : 1) * 3 * 4);
  L.part_l = o; o += al((size_t)(gb > 0 ? gb : 1) * 2 * 4);
  L.part_h = o; o += al((size_t)SEL_COPIES * SEL_HIST * 4);
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
  uint32_t* part_u = (uint32_t*)(ws + L.part_u);
  uint32_t* part_l = (uint32_t*)(ws + L.part_l);
  uint32_t* part_h = (uint32_t*)(ws + L.part_h);
  MpScal* sc = (MpScal*)(ws + L.scal);
  GaussOut go{(float*)(ws + L.Mhat), (float*)(ws + L.sde), (float*)(ws + L.U), (uint8_t*)(ws + L.obs)};
  float2* pk = (float2*)(ws + L.pk);
  const int K = fr->n_inst;
  const int nb = (int)((P + REG_TILE - 1) / REG_TILE);
  if (nb > 0)
    GS_LAUNCH(ctx, mp_region_kernel, dim3(nb), dim3(GS_BLOCK), 0, s, P, P, K, img->depth, tgt->depth, img->color,
              tgt->color, fr->instance_id, pp->beta_color, e, part, (int64_t)nb * (GS_BLOCK / 64));
  GS_LAUNCH(ctx, mp_region_final_kernel, dim3(1), dim3(MAXR * 64), 0, s, part, nb * (GS_BLOCK / 64), K,
            pp->lambda_e, pp->e_floor, pp->sigma_g, sc, out->judge);
  if (P > 0)
    GS_LAUNCH(ctx, mp_pixel_kernel, dim3((unsigned)((P + GS_BLOCK - 1) / GS_BLOCK)), dim3(GS_BLOCK), 0, s, P, K,
              e, fr->instance_id, fr->inst_prior, fr->inst_conf, fr->mlp_mp, pp->sigma_small, sc, Mp, out->e,
              tgt->depth, pk, out->judge);
  const unsigned gb = (unsigned)((n + GS_BLOCK - 1) / GS_BLOCK);
  if (n > 0)
    GS_LAUNCH(ctx, mp_gauss_kernel, dim3(gb), dim3(GS_BLOCK), 0, s, tab, proj->mean2d, proj->depth_key, pk, mp,
              pp->radius_px, pp->sigma_w, pp->lambda_u, pp->eps, go, part_u);
  GS_LAUNCH(ctx, mp_ureduce_kernel, dim3(1), dim3(1024), 0, s, part_u, (int)gb, sc, part_h);
  if (n > 0)
    GS_LAUNCH(ctx, mp_state_kernel, dim3(gb), dim3(GS_BLOCK), 0, s, tab, go, sc, pp->sigma_c, pp->lambda_u,
              pp->alpha_min, pp->alpha_max, pp->rho, fr->seg_updated, pp->mode, pp->u_norm, pp->logodds_eps,
              pp->logodds_max, mp, out->U_tilde, out->alpha);
  for (int pass = 0; pass < SEL_PASSES; ++pass) {
    GS_LAUNCH(ctx, mp_sel_hist_kernel, dim3(SEL_BLOCKS), dim3(GS_BLOCK), 0, s, n, tab.g_off[0], go.obs, mp,
              out->U_tilde, pass, sc, part_h);
    GS_LAUNCH(ctx, mp_sel_pick_kernel, dim3(1), dim3(1024), 0, s, pass, part_h, sc);
  }
  if (n > 0)
    GS_LAUNCH(ctx, mp_label_kernel, dim3(gb), dim3(GS_BLOCK), 0, s, tab, mp, pp->prune_above, sc, out->dynamic,
              out->prune, part_l);
  GS_LAUNCH(ctx, mp_stats_kernel, dim3(1), dim3(1024), 0, s, sc, part_l, (int)gb, out->stats);
  return gs_check_launch(ctx, "mp_update");
}
