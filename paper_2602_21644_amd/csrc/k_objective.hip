// The two further terms of the mapping objective (Sec. IV-D):
//
// gs_mp_regularizer: the MP-based motion consistency, Eq. (23)-(24),
//   lambda sum_k (1 - M_k) |mu_k - (R mu_prev_k + t)|^2, its gradient
//   2 lambda (1 - M_k)(mu_k - mu_hat_k) added into the mean gradient. One
//   thread per Gaussian, float64 loss partials per workgroup summed in a fixed
//   order by one more workgroup. HBM bound: 28 B read and 12 B read + written
//   per Gaussian.
//
// gs_edge_warp: the MP-guided edge-warp term, Eq. (25)-(26), for pairs of
//   views (i, j) of the batch. One thread per pixel u of frame i: the Sobel
//   slope of the observed depth, in float32 with a fixed operation order
//   (|(S_x, S_y)| / 8 above edge_thresh, 3x3 neighbourhood observed), decides
//   whether u is an edge pixel; only edge pixels go on: u is lifted with its
//   observed depth, carried by T_j T_i^-1 and projected with K_j (in double:
//   the pixels are few and the bilinear weights then match the reference
//   closely), frame j's rendered depth and static weight w^j = 1 - M/(1 - T)
//   are sampled bilinearly at u', and lambda huber(w (D_j(u') - D_i(u))) is
//   summed. The adjoint (w held constant) is added to frame j's depth adjoint
//   at the four neighbours (float atomics) and, through u', to the left pose
//   twists of both frames: per-workgroup float64 partials, summed per pair in
//   a fixed order by a one-workgroup kernel that walks the pairs in turn (two
//   pairs may share a view).
#include "gs_internal.h"

namespace {

constexpr int RG_PER = 4;  // Gaussians per thread
constexpr int RG_TILE = GS_BLOCK * RG_PER;

__global__ __launch_bounds__(GS_BLOCK) void mp_reg_kernel(int64_t n, const float* __restrict__ mean,
                                                          const float* __restrict__ prev, const float* __restrict__ mp,
                                                          float r00, float r01, float r02, float r10, float r11,
                                                          float r12, float r20, float r21, float r22, float t0,
                                                          float t1, float t2, int ident, float lam,
                                                          float* __restrict__ dmean, double* __restrict__ part) {
  __shared__ double s[GS_BLOCK / 64];
  const int64_t base = (int64_t)blockIdx.x * RG_TILE;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < RG_PER; ++q) {
    const int64_t k = base + q * GS_BLOCK + threadIdx.x;
    if (k >= n) continue;
    const float wb = 1.0f - mp[k];
    const float p0 = prev[k], p1 = prev[n + k], p2 = prev[2 * n + k];
    float h0 = p0, h1 = p1, h2 = p2;
    if (!ident) {
      h0 = r00 * p0 + r01 * p1 + r02 * p2 + t0;
      h1 = r10 * p0 + r11 * p1 + r12 * p2 + t1;
      h2 = r20 * p0 + r21 * p1 + r22 * p2 + t2;
    }
    const float d0 = mean[k] - h0, d1 = mean[n + k] - h1, d2 = mean[2 * n + k] - h2;
    acc += (double)wb * ((double)d0 * d0 + (double)d1 * d1 + (double)d2 * d2);
    const float g = 2.0f * lam * wb;
    dmean[k] += g * d0;
    dmean[n + k] += g * d1;
    dmean[2 * n + k] += g * d2;
  }
  acc = wave_sum_all_d(acc);
  if (__lane_id() == 63) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (double)lam * (s[0] + s[1] + s[2] + s[3]);
}

__global__ __launch_bounds__(GS_BLOCK) void sum_partials_kernel(const double* __restrict__ part, int64_t nb,
                                                                float* __restrict__ out) {
  __shared__ double s[GS_BLOCK / 64];
  double t = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += GS_BLOCK) t += part[b];
  t = wave_sum_all_d(t);
  if (__lane_id() == 63) s[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) *out = (float)(s[0] + s[1] + s[2] + s[3]);
}

// ---------------------------------------------------------------- edge warp
struct PairTab {
  int32_t i[GS_MAX_VIEWS], j[GS_MAX_VIEWS];
  int32_t np;
  int32_t nb;  // workgroups per pair (the largest frame i)
};

constexpr int EW_PART = 13;  // loss, then (rho, phi) of frame i, then of frame j

__device__ __forceinline__ float f_add(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ float f_mul(float a, float b) { return __fmul_rn(a, b); }

// Sobel slopes with every rounding spelled out: ((a + 2 b) + c) - ((d + 2 e) +
// f), times 1/8; then gx gx + gy gy, no fused multiply-add.
__device__ __forceinline__ float sobel_m2(const float* __restrict__ D, int64_t row, int W, int x) {
  const float* up = D + row - W;
  const float* mi = D + row;
  const float* dn = D + row + W;
  const float r = f_add(f_add(up[x + 1], f_mul(2.0f, mi[x + 1])), dn[x + 1]);
  const float l = f_add(f_add(up[x - 1], f_mul(2.0f, mi[x - 1])), dn[x - 1]);
  const float gx = f_mul(f_add(r, -l), 0.125f);
  const float b = f_add(f_add(dn[x - 1], f_mul(2.0f, dn[x])), dn[x + 1]);
  const float t = f_add(f_add(up[x - 1], f_mul(2.0f, up[x])), up[x + 1]);
  const float gy = f_mul(f_add(b, -t), 0.125f);
  return f_add(f_mul(gx, gx), f_mul(gy, gy));
}

__device__ __forceinline__ double static_w(float M, float T, float epsA) {
  const float A = 1.0f - T;
  return A > epsA ? (double)(1.0f - M / A) : 0.0;
}

__global__ __launch_bounds__(GS_BLOCK) void edge_warp_kernel(ViewTab tab, PairTab pt, const gs_camera* __restrict__ cams,
                                                             const float* __restrict__ Dobs,
                                                             const float* __restrict__ Drend,
                                                             const float* __restrict__ Mrend,
                                                             const float* __restrict__ Trend, float lam, float delta,
                                                             float thresh, float epsA, float* __restrict__ dD,
                                                             double* __restrict__ part) {
  __shared__ double s_red[EW_PART][GS_BLOCK / 64];
  const int pr = blockIdx.y;
  const int vi = pt.i[pr], vj = pt.j[pr];
  const int Wi = tab.W[vi], Hi = tab.H[vi], Wj = tab.W[vj], Hj = tab.H[vj];
  const int64_t p = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  double acc[EW_PART];
#pragma unroll
  for (int c = 0; c < EW_PART; ++c) acc[c] = 0.0;
  const int x = (int)(p % Wi), y = (int)(p / Wi);
  const float* Di = Dobs + tab.px_off[vi];
  bool edge = false;
  if (p < (int64_t)Wi * Hi && x > 0 && y > 0 && x < Wi - 1 && y < Hi - 1) {
    bool full = true;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) full = full && Di[(int64_t)(y + dy) * Wi + x + dx] > 0.f;
    if (full) edge = sobel_m2(Di, (int64_t)y * Wi, Wi, x) > f_mul(thresh, thresh);
  }
  if (edge) {
    const gs_camera& ci = cams[vi];
    const gs_camera& cj = cams[vj];
    const double d = (double)Di[(int64_t)y * Wi + x];
    // camera i -> world -> camera j
    const double X0 = d * ((double)x - ci.cx) / ci.fx, X1 = d * ((double)y - ci.cy) / ci.fy, X2 = d;
    const float* Ti = ci.T_cw;
    const float* Tj = cj.T_cw;
    const double a0 = X0 - Ti[3], a1 = X1 - Ti[7], a2 = X2 - Ti[11];
    const double w0 = (double)Ti[0] * a0 + (double)Ti[4] * a1 + (double)Ti[8] * a2;
    const double w1 = (double)Ti[1] * a0 + (double)Ti[5] * a1 + (double)Ti[9] * a2;
    const double w2 = (double)Ti[2] * a0 + (double)Ti[6] * a1 + (double)Ti[10] * a2;
    const double P0 = (double)Tj[0] * w0 + (double)Tj[1] * w1 + (double)Tj[2] * w2 + Tj[3];
    const double P1 = (double)Tj[4] * w0 + (double)Tj[5] * w1 + (double)Tj[6] * w2 + Tj[7];
    const double P2 = (double)Tj[8] * w0 + (double)Tj[9] * w1 + (double)Tj[10] * w2 + Tj[11];
    const double ux = (double)cj.fx * P0 / P2 + cj.cx, uy = (double)cj.fy * P1 / P2 + cj.cy;
    const double x0 = floor(ux), y0 = floor(uy);
    if (P2 > (double)cj.z_near && x0 >= 0.0 && x0 + 1.0 <= Wj - 1 && y0 >= 0.0 && y0 + 1.0 <= Hj - 1) {
      const double fx = ux - x0, fy = uy - y0;
      const int64_t q00 = tab.px_off[vj] + (int64_t)y0 * Wj + (int64_t)x0, q01 = q00 + 1, q10 = q00 + Wj,
                    q11 = q10 + 1;
      const double D00 = Drend[q00], D01 = Drend[q01], D10 = Drend[q10], D11 = Drend[q11];
      const double b00 = (1 - fx) * (1 - fy), b01 = fx * (1 - fy), b10 = (1 - fx) * fy, b11 = fx * fy;
      const double Ds = b00 * D00 + b01 * D01 + b10 * D10 + b11 * D11;
      const double ws = b00 * static_w(Mrend[q00], Trend[q00], epsA) + b01 * static_w(Mrend[q01], Trend[q01], epsA) +
                        b10 * static_w(Mrend[q10], Trend[q10], epsA) + b11 * static_w(Mrend[q11], Trend[q11], epsA);
      const double r = ws * (Ds - d);
      const double ar = fabs(r);
      acc[0] = lam * (ar <= delta ? 0.5 * r * r : delta * (ar - 0.5 * delta));
      const double g = lam * fmin(fmax(r, -(double)delta), (double)delta) * ws;
      atomicAdd(dD + q00, (float)(g * b00));
      atomicAdd(dD + q01, (float)(g * b01));
      atomicAdd(dD + q10, (float)(g * b10));
      atomicAdd(dD + q11, (float)(g * b11));
      // through u' (w held constant)
      const double gux = g * ((1 - fy) * (D01 - D00) + fy * (D11 - D10));
      const double guy = g * ((1 - fx) * (D10 - D00) + fx * (D11 - D01));
      const double gP0 = gux * cj.fx / P2, gP1 = guy * cj.fy / P2;
      const double gP2 = -(gux * cj.fx * P0 + guy * cj.fy * P1) / (P2 * P2);
      // frame j: rho += gP, phi += P x gP
      acc[7] = gP0;
      acc[8] = gP1;
      acc[9] = gP2;
      acc[10] = P1 * gP2 - P2 * gP1;
      acc[11] = P2 * gP0 - P0 * gP2;
      acc[12] = P0 * gP1 - P1 * gP0;
      // frame i: q = R_ji^T gP = R_i R_j^T gP; rho -= q, phi -= X x q
      const double v0 = (double)Tj[0] * gP0 + (double)Tj[4] * gP1 + (double)Tj[8] * gP2;
      const double v1 = (double)Tj[1] * gP0 + (double)Tj[5] * gP1 + (double)Tj[9] * gP2;
      const double v2 = (double)Tj[2] * gP0 + (double)Tj[6] * gP1 + (double)Tj[10] * gP2;
      const double q0 = (double)Ti[0] * v0 + (double)Ti[1] * v1 + (double)Ti[2] * v2;
      const double q1 = (double)Ti[4] * v0 + (double)Ti[5] * v1 + (double)Ti[6] * v2;
      const double q2 = (double)Ti[8] * v0 + (double)Ti[9] * v1 + (double)Ti[10] * v2;
      acc[1] = -q0;
      acc[2] = -q1;
      acc[3] = -q2;
      acc[4] = -(X1 * q2 - X2 * q1);
      acc[5] = -(X2 * q0 - X0 * q2);
      acc[6] = -(X0 * q1 - X1 * q0);
    }
  }
  // every pixel of the block has run the same reductions: sums in a fixed order
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < EW_PART; ++c) {
    const double t = wave_sum_all_d(acc[c]);
    if (__lane_id() == 63) s_red[c][w] = t;
  }
  __syncthreads();
  if (threadIdx.x < EW_PART) {
    const int c = threadIdx.x;
    part[((int64_t)pr * pt.nb + blockIdx.x) * EW_PART + c] = s_red[c][0] + s_red[c][1] + s_red[c][2] + s_red[c][3];
  }
}

// One workgroup: the pairs in turn, each pair's workgroup partials summed in a
// fixed order; the loss per pair, the pose adjoints added to both views.
__global__ __launch_bounds__(GS_BLOCK) void edge_warp_final_kernel(PairTab pt, const double* __restrict__ part,
                                                                   float* __restrict__ loss,
                                                                   float* __restrict__ dpose) {
  __shared__ double s[EW_PART][GS_BLOCK / 64];
  for (int pr = 0; pr < pt.np; ++pr) {
    double acc[EW_PART];
#pragma unroll
    for (int c = 0; c < EW_PART; ++c) acc[c] = 0.0;
    for (int b = threadIdx.x; b < pt.nb; b += GS_BLOCK) {
      const double* r = part + ((int64_t)pr * pt.nb + b) * EW_PART;
#pragma unroll
      for (int c = 0; c < EW_PART; ++c) acc[c] += r[c];
    }
#pragma unroll
    for (int c = 0; c < EW_PART; ++c) {
      const double t = wave_sum_all_d(acc[c]);
      if (__lane_id() == 63) s[c][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot[EW_PART];
#pragma unroll
      for (int c = 0; c < EW_PART; ++c) tot[c] = s[c][0] + s[c][1] + s[c][2] + s[c][3];
      loss[pr] = (float)tot[0];
      if (dpose) {
        for (int c = 0; c < 6; ++c) dpose[pt.i[pr] * 6 + c] += (float)tot[1 + c];
        for (int c = 0; c < 6; ++c) dpose[pt.j[pr] * 6 + c] += (float)tot[7 + c];
      }
    }
    __syncthreads();
  }
}

}  // namespace

size_t mp_reg_ws_bytes(int64_t n) { return (size_t)((n + RG_TILE - 1) / RG_TILE + 1) * 8; }

gs_status launch_mp_reg(gs_ctx* ctx, int64_t n, const float* mean, const float* prev, const float* mp, const float* T,
                        float lam, float* loss, float* dmean, double* part, hipStream_t s) {
  const int64_t nb = (n + RG_TILE - 1) / RG_TILE;
  float r[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
  if (T)
    for (int i = 0; i < 12; ++i) r[i] = T[i];
  const int ident = T ? 0 : 1;
  if (nb > 0)
    GS_LAUNCH(ctx, mp_reg_kernel, dim3((unsigned)nb), dim3(GS_BLOCK), 0, s, n, mean, prev, mp, r[0], r[1], r[2], r[4],
              r[5], r[6], r[8], r[9], r[10], r[3], r[7], r[11], ident, lam, dmean, part);
  GS_LAUNCH(ctx, sum_partials_kernel, dim3(1), dim3(GS_BLOCK), 0, s, part, nb, loss);
  return gs_check_launch(ctx, "mp_regularizer");
}

static int edge_blocks(const ViewTab& tab, const gs_edge_pair* pairs, int np) {
  int64_t mx = 0;
  for (int k = 0; k < np; ++k) {
    const int v = pairs[k].i;
    const int64_t px = (int64_t)tab.W[v] * tab.H[v];
    mx = px > mx ? px : mx;
  }
  return (int)((mx + GS_BLOCK - 1) / GS_BLOCK);
}

size_t edge_warp_ws_bytes(const ViewTab& tab, int32_t n_pairs) {
  int64_t mx = 0;
  for (int v = 0; v < tab.nv; ++v) mx = (int64_t)tab.W[v] * tab.H[v] > mx ? (int64_t)tab.W[v] * tab.H[v] : mx;
  return (size_t)n_pairs * (size_t)((mx + GS_BLOCK - 1) / GS_BLOCK) * EW_PART * 8;
}

gs_status launch_edge_warp(gs_ctx* ctx, const ViewTab& tab, const gs_camera* cams, const gs_image* img,
                           const gs_target* tgt, const gs_edge_pair* pairs, int32_t np, const gs_edge_params* ep,
                           float* loss, float* ddepth, float* dpose, double* part, hipStream_t s) {
  PairTab pt{};
  pt.np = np;
  for (int k = 0; k < np; ++k) {
    pt.i[k] = pairs[k].i;
    pt.j[k] = pairs[k].j;
  }
  pt.nb = edge_blocks(tab, pairs, np);
  if (np == 0) return GS_OK;
  GS_LAUNCH(ctx, edge_warp_kernel, dim3((unsigned)pt.nb, (unsigned)np), dim3(GS_BLOCK), 0, s, tab, pt, cams,
            tgt->depth, img->depth, img->mp, img->T, ep->lambda, ep->delta, ep->edge_thresh, ep->eps_A, ddepth, part);
  GS_LAUNCH(ctx, edge_warp_final_kernel, dim3(1), dim3(GS_BLOCK), 0, s, pt, part, loss, dpose);
  return gs_check_launch(ctx, "edge_warp");
}
