// EWA projection of one Gaussian in float32, shared by the projection kernel
// and the projection adjoint (which needs the intermediates).
#pragma once

#include "gs_internal.h"

struct ProjF {
  bool kept;
  float px, py, pz;       // camera-space mean
  float qn[4], qinv;      // unit quaternion and 1/|q|
  float Rq[3][3];         // Gaussian rotation
  float S[3];             // exp(log_scale)
  float T1[3][3];         // R * Rq * diag(S): camera-space square root of the covariance
  float j00, j02, j11, j12;
  float JT[2][3];         // J * T1
  float a, b, c, det;     // 2D covariance (with low-pass) and determinant
  float k1, k2, k3;       // conic
  float ux, uy;
  float o;
  float extent;
};

__device__ __forceinline__ bool finitef_(float x) { return __builtin_isfinite(x); }

__device__ __forceinline__ void quat_rot(const float q[4], float R[3][3]) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1.f - 2.f * (y * y + z * z); R[0][1] = 2.f * (x * y - w * z); R[0][2] = 2.f * (x * z + w * y);
  R[1][0] = 2.f * (x * y + w * z); R[1][1] = 1.f - 2.f * (x * x + z * z); R[1][2] = 2.f * (y * z - w * x);
  R[2][0] = 2.f * (x * z - w * y); R[2][1] = 2.f * (y * z + w * x); R[2][2] = 1.f - 2.f * (x * x + y * y);
}

// cam: the view's camera; m, ls, q, opl: the Gaussian's parameters. No
// multiply-add is fused here, so every kernel that inlines this function
// (the projection, the prefix binning, the projection adjoint) rounds the
// record of a Gaussian alike: the full and the prefix lists then composite
// bit-identical records.
__device__ __forceinline__ ProjF project_f(const gs_camera& cam, const float m[3], const float ls[3],
                                           const float q[4], float opl) {
#pragma clang fp contract(off)
  ProjF P;
  P.kept = false;
  bool fin = finitef_(m[0]) && finitef_(m[1]) && finitef_(m[2]) && finitef_(ls[0]) && finitef_(ls[1]) &&
             finitef_(ls[2]) && finitef_(q[0]) && finitef_(q[1]) && finitef_(q[2]) && finitef_(q[3]) &&
             finitef_(opl);
  const float* T = cam.T_cw;
  P.px = T[0] * m[0] + T[1] * m[1] + T[2] * m[2] + T[3];
  P.py = T[4] * m[0] + T[5] * m[1] + T[6] * m[2] + T[7];
  // camera z with every rounding spelled out: it orders the Gaussians (the
  // sort key is its bit pattern) and decides the near-plane cull
  P.pz = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(T[8], m[0]), __fmul_rn(T[9], m[1])), __fmul_rn(T[10], m[2])), T[11]);
  if (!fin || !(P.pz > cam.z_near)) return P;
  const float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  if (!(qq > 0.f)) return P;
  P.qinv = 1.0f / sqrtf(qq);
  for (int i = 0; i < 4; ++i) P.qn[i] = q[i] * P.qinv;
  quat_rot(P.qn, P.Rq);
  for (int i = 0; i < 3; ++i) P.S[i] = __expf(ls[i]);
  // T1 = R_cw * Rq * diag(S)
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      P.T1[i][j] = (T[4 * i + 0] * P.Rq[0][j] + T[4 * i + 1] * P.Rq[1][j] + T[4 * i + 2] * P.Rq[2][j]) * P.S[j];
  const float iz = 1.0f / P.pz;
  P.j00 = cam.fx * iz;
  P.j11 = cam.fy * iz;
  P.j02 = -cam.fx * P.px * iz * iz;
  P.j12 = -cam.fy * P.py * iz * iz;
  for (int j = 0; j < 3; ++j) {
    P.JT[0][j] = P.j00 * P.T1[0][j] + P.j02 * P.T1[2][j];
    P.JT[1][j] = P.j11 * P.T1[1][j] + P.j12 * P.T1[2][j];
  }
  P.a = P.JT[0][0] * P.JT[0][0] + P.JT[0][1] * P.JT[0][1] + P.JT[0][2] * P.JT[0][2] + 0.3f;
  P.b = P.JT[0][0] * P.JT[1][0] + P.JT[0][1] * P.JT[1][1] + P.JT[0][2] * P.JT[1][2];
  P.c = P.JT[1][0] * P.JT[1][0] + P.JT[1][1] * P.JT[1][1] + P.JT[1][2] * P.JT[1][2] + 0.3f;
  P.det = P.a * P.c - P.b * P.b;
  if (!(P.det > 0.f)) return P;
  const float idet = 1.0f / P.det;
  P.k1 = P.c * idet;
  P.k2 = -P.b * idet;
  P.k3 = P.a * idet;
  P.ux = cam.fx * P.px * iz + cam.cx;
  P.uy = cam.fy * P.py * iz + cam.cy;
  P.o = 1.0f / (1.0f + __expf(-opl));
  if (!(P.o >= GS_ALPHA_MIN)) return P;
  const float h = 0.5f * (P.a - P.c);
  const float lmax = 0.5f * (P.a + P.c) + sqrtf(h * h + P.b * P.b);
  P.extent = sqrtf(2.0f * __logf(255.0f * P.o) * lmax);
  P.kept = true;
  return P;
}

// The tile rect of a projected Gaussian: pixels floor(u) -/+ ceil(extent),
// clipped to the view's tile grid; false when the Gaussian was culled or the
// rect misses the grid. Gaussians whose projected mean or radius exceed 1e7 px
// are treated as off-screen (the integer pixel arithmetic needs exact floats).
__device__ __forceinline__ bool tile_rect_of(const ProjF& P, int gx, int gy, int2& rc, int& rr) {
  rr = 0;
  rc = make_int2((int)(uint16_t)1 | ((int)(uint16_t)1 << 16), 0);  // empty: x0 = 1 > x1 = 0
  if (!P.kept) return false;
  const float rf = ceilf(P.extent);
  if (!(fabsf(P.ux) < 1e7f && fabsf(P.uy) < 1e7f && rf < 1e7f)) return false;
  rr = (int)rf;
  const int ix = (int)floorf(P.ux), iy = (int)floorf(P.uy);
  const int x0 = max(0, (ix - rr) >> 4), x1 = min(gx - 1, (ix + rr) >> 4);
  const int y0 = max(0, (iy - rr) >> 4), y1 = min(gy - 1, (iy + rr) >> 4);
  if (x0 > x1 || y0 > y1) return false;
  rc = make_int2((x0 & 0xFFFF) | (y0 << 16), (x1 & 0xFFFF) | (y1 << 16));
  return true;
}

// A cheap test that never rejects a Gaussian the exact projection keeps: the
// depth key (the same float32 camera z as project_f), the same near-plane and
// opacity culls, and a tile rect from a bound on the footprint: the largest
// eigenvalue of J R Sigma R^T J^T + 0.3 I is at most |J|_F^2 exp(2 max
// log_scale) + 0.3, widened by 0.1% and one pixel. Returns the key, or
// 0xFFFFFFFF when even the bound misses the view.
__device__ __forceinline__ uint32_t screen_key(const gs_camera& cam, const float m[3], const float ls[3], float opl,
                                               int gx, int gy) {
  const float* T = cam.T_cw;
  const float pz = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(T[8], m[0]), __fmul_rn(T[9], m[1])), __fmul_rn(T[10], m[2])),
                             T[11]);
  if (!(pz > cam.z_near)) return 0xFFFFFFFFu;  // also NaN
  const float o = 1.0f / (1.0f + __expf(-opl));
  if (!(o >= GS_ALPHA_MIN)) return 0xFFFFFFFFu;
  const float px = T[0] * m[0] + T[1] * m[1] + T[2] * m[2] + T[3];
  const float py = T[4] * m[0] + T[5] * m[1] + T[6] * m[2] + T[7];
  const float iz = 1.0f / pz;
  const float ux = cam.fx * px * iz + cam.cx, uy = cam.fy * py * iz + cam.cy;
  const float ax = cam.fx * iz, ay = cam.fy * iz, bx = ax * px * iz, by = ay * py * iz;
  const float jf2 = ax * ax + bx * bx + ay * ay + by * by;
  const float smax = fmaxf(fmaxf(ls[0], ls[1]), ls[2]);
  const float lb = (jf2 * __expf(2.0f * smax) + 0.3f) * 1.001f;
  const float ext = sqrtf(2.0f * __logf(255.0f * o) * lb) * 1.001f + 1.0f;
  const float rf = ceilf(ext);
  // outside the integer range of the exact test: keep (never wrongly culled)
  if (!(fabsf(ux) < 1e7f && fabsf(uy) < 1e7f && rf < 1e7f)) return __float_as_uint(pz);
  const int r = (int)rf;
  const int ix = (int)floorf(ux), iy = (int)floorf(uy);
  const int x0 = max(0, (ix - r) >> 4), x1 = min(gx - 1, (ix + r) >> 4);
  const int y0 = max(0, (iy - r) >> 4), y1 = min(gy - 1, (iy + r) >> 4);
  return (x0 <= x1 && y0 <= y1) ? __float_as_uint(pz) : 0xFFFFFFFFu;
}

// Gaussian parameter planes, passed by value to the compositing kernels.
struct GaussSrc {
  const float *mean, *log_scale, *quat, *opl, *color, *mp;
  int64_t n;
};

// The compositing record of packed Gaussian gk seen by `cam`: (u_x, u_y, z,
// opacity), (conic in base-2 exponent units, mp), (rgb, 0). Computed by the
// same project_f as the projection kernel, so it matches the record the tile
// rect came from.
__device__ __forceinline__ void render_record(const gs_camera& cam, const GaussSrc& g, int64_t gk, float4& a,
                                              float4& b, float4& c) {
  const int64_t N = g.n;
  const float m[3] = {g.mean[gk], g.mean[N + gk], g.mean[2 * N + gk]};
  const float ls[3] = {g.log_scale[gk], g.log_scale[N + gk], g.log_scale[2 * N + gk]};
  const float q[4] = {g.quat[gk], g.quat[N + gk], g.quat[2 * N + gk], g.quat[3 * N + gk]};
  const ProjF P = project_f(cam, m, ls, q, g.opl[gk]);
  a = make_float4(P.ux, P.uy, P.pz, P.o);
  b = make_float4(gs_conic_scale_diag(P.k1), gs_conic_scale_off(P.k2), gs_conic_scale_diag(P.k3), g.mp[gk]);
  c = make_float4(g.color[gk], g.color[N + gk], g.color[2 * N + gk], 0.f);
}
