// gs_adam_step and gs_pose_update: the optimiser steps of the joint
// optimisation of Gaussians and poses.
//
// Adam: one launch over all groups; each thread updates 4 consecutive
// elements of a group with float4 loads where the group's arrays allow it.
// Pose update: one thread per view, in double precision: the SE(3)
// exponential of the twist (Rodrigues' formula for the rotation, the left
// Jacobian for the translation, Taylor series below a small angle), the
// left composition with T_cw and a Gram-Schmidt re-orthonormalisation.
#include "gs_internal.h"

namespace {

struct AdamTab {
  float* param[GS_ADAM_MAX_GROUPS];
  const float* grad[GS_ADAM_MAX_GROUPS];
  float* m[GS_ADAM_MAX_GROUPS];
  float* v[GS_ADAM_MAX_GROUPS];
  int64_t n[GS_ADAM_MAX_GROUPS];
  int64_t blk0[GS_ADAM_MAX_GROUPS + 1];  // first block of each group
  float lr[GS_ADAM_MAX_GROUPS];
  int ng;
  float b1, b2, eps, c1, c2;  // c1 = 1 / (1 - b1^step), c2 = 1 / (1 - b2^step)
  int32_t* step_dev;          // when set, c1 and c2 come from the device step count
  int bump;                   // one-workgroup launch: advance *step_dev by one first
  int small;                  // every group fits one tile: one workgroup does them all
};

constexpr int ADAM_PER = 4;
constexpr int ADAM_TILE = GS_BLOCK * ADAM_PER;

__device__ __forceinline__ void adam_one(const AdamTab& t, float c1, float c2, float& p, float g, float& m,
                                         float& v, float lr) {
  m = t.b1 * m + (1.0f - t.b1) * g;
  v = t.b2 * v + (1.0f - t.b2) * g * g;
  const float mh = m * c1, vh = v * c2;
  p -= lr * mh / (sqrtf(vh) + t.eps);
}

// Advances the device step count of a multi-workgroup Adam launch.
__global__ void step_advance_kernel(int32_t* step) { *step += 1; }

// One tile of group gi: ADAM_PER elements per thread from element i0.
__device__ __forceinline__ void adam_tile(const AdamTab& t, float c1, float c2, int gi, int64_t i0) {
  const int64_t n = t.n[gi];
  if (i0 >= n) return;
  float* P = t.param[gi];
  const float* G = t.grad[gi];
  float* Mv = t.m[gi];
  float* Vv = t.v[gi];
  const float lr = t.lr[gi];
  const bool vec = i0 + ADAM_PER <= n && ((((uintptr_t)P | (uintptr_t)G | (uintptr_t)Mv | (uintptr_t)Vv) & 15) == 0);
  if (vec) {
    float4 p = *(float4*)(P + i0), m = *(float4*)(Mv + i0), v = *(float4*)(Vv + i0);
    const float4 g = *(const float4*)(G + i0);
    adam_one(t, c1, c2, p.x, g.x, m.x, v.x, lr);
    adam_one(t, c1, c2, p.y, g.y, m.y, v.y, lr);
    adam_one(t, c1, c2, p.z, g.z, m.z, v.z, lr);
    adam_one(t, c1, c2, p.w, g.w, m.w, v.w, lr);
    *(float4*)(P + i0) = p;
    *(float4*)(Mv + i0) = m;
    *(float4*)(Vv + i0) = v;
  } else {
    for (int64_t i = i0; i < n && i < i0 + ADAM_PER; ++i) {
      float p = P[i], m = Mv[i], v = Vv[i];
      adam_one(t, c1, c2, p, G[i], m, v, lr);
      P[i] = p;
      Mv[i] = m;
      Vv[i] = v;
    }
  }
}

__global__ __launch_bounds__(GS_BLOCK) void adam_kernel(AdamTab t) {
  float c1 = t.c1, c2 = t.c2;
  if (t.step_dev) {
    const int32_t s0 = *t.step_dev + t.bump;
    const double s = (double)max(1, s0);
    c1 = (float)(1.0 / (1.0 - pow((double)t.b1, s)));
    c2 = (float)(1.0 / (1.0 - pow((double)t.b2, s)));
    if (t.bump) {
      // the only workgroup: every thread has read the count before it moves
      __syncthreads();
      if (threadIdx.x == 0) *t.step_dev = s0;
    }
  }
  if (t.small) {
    // every group fits one tile: this single workgroup walks them in turn
    for (int gi = 0; gi < t.ng; ++gi) adam_tile(t, c1, c2, gi, (int64_t)threadIdx.x * ADAM_PER);
    return;
  }
  const int64_t blk = blockIdx.x;
  int gi = 0;
  while (gi + 1 < t.ng && blk >= t.blk0[gi + 1]) ++gi;
  adam_tile(t, c1, c2, gi, (blk - t.blk0[gi]) * ADAM_TILE + (int64_t)threadIdx.x * ADAM_PER);
}

// T <- Exp(delta) T for view v; delta zeroed.
__global__ void pose_update_kernel(int nv, gs_camera* __restrict__ cams, float* __restrict__ delta) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double rho[3], phi[3];
  for (int i = 0; i < 3; ++i) {
    rho[i] = delta[6 * v + i];
    phi[i] = delta[6 * v + 3 + i];
  }
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const double th = sqrt(th2);
  double A, B, C;  // sin(th)/th, (1 - cos th)/th^2, (th - sin th)/th^3
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  // K = [phi]x, K2 = K K
  const double K[3][3] = {{0.0, -phi[2], phi[1]}, {phi[2], 0.0, -phi[0]}, {-phi[1], phi[0], 0.0}};
  double K2[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
  double Rd[3][3], Vd[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double I = i == j ? 1.0 : 0.0;
      Rd[i][j] = I + A * K[i][j] + B * K2[i][j];
      Vd[i][j] = I + B * K[i][j] + C * K2[i][j];
    }
  double td[3];
  for (int i = 0; i < 3; ++i) td[i] = Vd[i][0] * rho[0] + Vd[i][1] * rho[1] + Vd[i][2] * rho[2];
  float* T = cams[v].T_cw;
  double R[3][3], t[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) R[i][j] = T[4 * i + j];
    t[i] = T[4 * i + 3];
  }
  double Rn[3][3], tn[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) Rn[i][j] = Rd[i][0] * R[0][j] + Rd[i][1] * R[1][j] + Rd[i][2] * R[2][j];
    tn[i] = Rd[i][0] * t[0] + Rd[i][1] * t[1] + Rd[i][2] * t[2] + td[i];
  }
  // Gram-Schmidt on the rows keeps R a rotation under float storage
  for (int i = 0; i < 3; ++i) {
    for (int k = 0; k < i; ++k) {
      const double d = Rn[i][0] * Rn[k][0] + Rn[i][1] * Rn[k][1] + Rn[i][2] * Rn[k][2];
      for (int j = 0; j < 3; ++j) Rn[i][j] -= d * Rn[k][j];
    }
    const double nrm = sqrt(Rn[i][0] * Rn[i][0] + Rn[i][1] * Rn[i][1] + Rn[i][2] * Rn[i][2]);
    for (int j = 0; j < 3; ++j) Rn[i][j] /= nrm;
  }
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) T[4 * i + j] = (float)Rn[i][j];
    T[4 * i + 3] = (float)tn[i];
  }
  for (int i = 0; i < 6; ++i) delta[6 * v + i] = 0.f;
}

}  // namespace

extern "C" {

gs_status gs_adam_step(gs_ctx* ctx, const gs_adam_group* groups, int32_t n_groups, const gs_adam_params* params,
                       void* stream) {
  if (!ctx || !groups || !params) return gs_fail(ctx, GS_E_ARG, "null argument");
  if (n_groups < 1 || n_groups > GS_ADAM_MAX_GROUPS) return gs_fail(ctx, GS_E_ARG, "n_groups must be 1..%d",
                                                                     GS_ADAM_MAX_GROUPS);
  if (params->step < 1 && !params->step_dev) return gs_fail(ctx, GS_E_ARG, "step must be >= 1");
  if (!(params->beta1 >= 0.f && params->beta1 < 1.f && params->beta2 >= 0.f && params->beta2 < 1.f &&
        params->eps > 0.f))
    return gs_fail(ctx, GS_E_ARG, "beta1, beta2 in [0, 1) and eps > 0");
  AdamTab t;
  t.ng = n_groups;
  t.b1 = params->beta1;
  t.b2 = params->beta2;
  t.eps = params->eps;
  const double st = params->step < 1 ? 1.0 : (double)params->step;
  t.c1 = (float)(1.0 / (1.0 - pow((double)params->beta1, st)));
  t.c2 = (float)(1.0 / (1.0 - pow((double)params->beta2, st)));
  t.step_dev = params->step_dev;
  t.bump = 0;
  t.small = 0;
  int64_t blocks = 0;
  for (int i = 0; i < n_groups; ++i) {
    const gs_adam_group& g = groups[i];
    if (g.n < 0) return gs_fail(ctx, GS_E_ARG, "group %d: n < 0", i);
    if (g.n > 0 && (!g.param || !g.grad || !g.m || !g.v)) return gs_fail(ctx, GS_E_ARG, "group %d: NULL array", i);
    t.param[i] = g.param;
    t.grad[i] = g.grad;
    t.m[i] = g.m;
    t.v[i] = g.v;
    t.n[i] = g.n;
    t.lr[i] = g.lr;
    t.blk0[i] = blocks;
    blocks += (g.n + ADAM_TILE - 1) / ADAM_TILE;
  }
  t.blk0[n_groups] = blocks;
  if (blocks > 1 && blocks == n_groups) {
    // small groups (a pose twist): one workgroup walks all of them
    t.small = 1;
    blocks = 1;
  }
  if (params->advance && params->step_dev) {
    if (blocks == 1)
      t.bump = 1;  // the kernel advances the count itself
    else
      GS_LAUNCH(ctx, step_advance_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream, params->step_dev);
  }
  if (blocks == 0) return gs_check_launch(ctx, "adam_step");
  GS_LAUNCH(ctx, adam_kernel, dim3((unsigned)blocks), dim3(GS_BLOCK), 0, (hipStream_t)stream, t);
  return gs_check_launch(ctx, "adam_step");
}

gs_status gs_pose_update(gs_ctx* ctx, int32_t n_views, gs_camera* cams, float* delta, void* stream) {
  if (!ctx || !cams || !delta) return gs_fail(ctx, GS_E_ARG, "null argument");
  if (n_views < 1 || n_views > GS_MAX_VIEWS) return gs_fail(ctx, GS_E_ARG, "n_views must be 1..%d", GS_MAX_VIEWS);
  GS_LAUNCH(ctx, pose_update_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, n_views, cams, delta);
  return gs_check_launch(ctx, "pose_update");
}

}  // extern "C"
