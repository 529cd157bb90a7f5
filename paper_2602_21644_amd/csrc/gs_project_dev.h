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

// cam: the view's camera; m, ls, q, opl: the Gaussian's parameters.
__device__ __forceinline__ ProjF project_f(const gs_camera& cam, const float m[3], const float ls[3],
                                           const float q[4], float opl) {
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
