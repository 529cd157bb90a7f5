// Second part of gs_render_bwd: per-Gaussian adjoint of the projection.
//
// One thread per Gaussian (all scenes); it visits every view of its scene,
// reads the 2D adjoint the tile pass accumulated for that (view, Gaussian)
// record (the sum of its per-XCD copies, gathered by the whole wave) only
// when the record was touched, chains it through the projection in float32
// and sums the parameter gradients over views in registers. Read records are
// reset to zero so the scratch stays zero-filled between calls.
// The grid is as many blocks as the device holds at once; block b takes the
// groups of GS_BLOCK Gaussians b, b + grid, ... Most Gaussians of a large
// scene are never composited, so a wave loads the touched flags of its next
// group while it works on the current one, and a wave without any touched
// record only stores zero gradients (nothing at all when accumulating), with
// no block barrier. Pose-twist partials are summed per wave into LDS, then
// per block, and the block partials in a fixed order by a second kernel
// (deterministic).
//
// The chain works with the camera-space square root T1 = R Rq diag(S) of the
// covariance (cov2D = (J T1)(J T1)^T + 0.3 I), a different route from the
// covariance-space derivation of the CPU reference.
#include "gs_project_dev.h"

namespace {

constexpr int kMaxCopies = 8;  // largest "bwd_copies"

// Views of the scene in which Gaussian gk has a touched record, as a bit mask.
__device__ __forceinline__ uint32_t touched_views(const ViewTab& tab, const uint8_t* __restrict__ touched,
                                                  int64_t gk) {
  uint32_t h = 0u;
  for (int v = 0; v < tab.nv; ++v) {
    const int64_t k = gk - tab.g_off[v];
    if (gk < tab.ng && k >= 0 && k < tab.n[v] && touched[tab.r_off[v] + k] != 0) h |= 1u << v;
  }
  return h;
}

// The 2D adjoint of record r, summed over its `copies` accumulators (layout
// [copy][record][10]) and reset to zero, for every lane with hit set. The
// whole wave gathers one record at a time: lane 5 x + k loads float2 k of
// copy x, a fixed shuffle tree sums the copies, and the owning lane takes the
// five sums. Wave-uniform control flow; lanes without a hit get zeros.
__device__ __forceinline__ void gather_adjoint(bool hit, int64_t r, int64_t M, int copies, float* __restrict__ g2d,
                                               float (&a)[10]) {
  const int lane = __lane_id();
#pragma unroll
  for (int c = 0; c < 10; ++c) a[c] = 0.f;
  uint64_t m = __ballot(hit);
  const int cp = lane / 5, kk = lane - 5 * (lane / 5);
  while (m) {
    const int src = __ffsll((long long)m) - 1;
    m &= m - 1;
    const int64_t rs = __shfl(r, src, 64);
    float2 t = make_float2(0.f, 0.f);
    if (cp < copies) {
      float2* p = reinterpret_cast<float2*>(g2d + ((int64_t)cp * M + rs) * 10) + kk;
      t = *p;
      *p = make_float2(0.f, 0.f);
    }
    // copies x and x + 4, then x + 2, then x + 1 (zeros past `copies`)
#pragma unroll
    for (int off = 20; off >= 5; off >>= 1) {
      t.x += __shfl_down(t.x, off, 64);
      t.y += __shfl_down(t.y, off, 64);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const float x = __shfl(t.x, k, 64), y = __shfl(t.y, k, 64);
      if (lane == src) {
        a[2 * k] = x;
        a[2 * k + 1] = y;
      }
    }
  }
}

__global__ __launch_bounds__(GS_BLOCK) void bwd_project_kernel(
    ViewTab tab, const gs_camera* __restrict__ cams, const float* __restrict__ mean,
    const float* __restrict__ log_scale, const float* __restrict__ quat, const float* __restrict__ opl,
    float* __restrict__ g2d, uint8_t* __restrict__ touched, float* __restrict__ d_mean,
    float* __restrict__ d_ls, float* __restrict__ d_quat, float* __restrict__ d_opl, float* __restrict__ d_color,
    float* __restrict__ pose_part, int pstride, int pose_only, int accumulate, int copies) {
  __shared__ float s_pose[GS_BLOCK / 64][GS_MAX_VIEWS * 6];  // per-wave pose sums
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int64_t N = tab.ng;
  const int64_t M = tab.nrec;
  for (int i = lane; i < tab.nv * 6; i += 64) s_pose[wv][i] = 0.f;
  __syncthreads();
  const int64_t ngroups = (N + GS_BLOCK - 1) / GS_BLOCK;
  uint32_t hnext = touched_views(tab, touched, (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x);
#pragma unroll 1
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const uint32_t hg = hnext;
    hnext = touched_views(tab, touched, (grp + gridDim.x) * GS_BLOCK + threadIdx.x);
    const int64_t gk = grp * GS_BLOCK + threadIdx.x;
    const bool valid = gk < N;
    float gm[3] = {0, 0, 0}, gl[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.f, gc[3] = {0, 0, 0};
    if (__ballot(hg != 0u) != 0) {
      // parameters of touched Gaussians, in flight during the adjoint gather
      float m[3] = {0, 0, 0}, ls[3] = {0, 0, 0}, q[4] = {1, 0, 0, 0}, op = 0.f;
      if (hg != 0u) {
        for (int c = 0; c < 3; ++c) {
          m[c] = mean[c * N + gk];
          ls[c] = log_scale[c * N + gk];
        }
        for (int c = 0; c < 4; ++c) q[c] = quat[c * N + gk];
        op = opl[gk];
      }
      for (int v = 0; v < tab.nv; ++v) {
        float pv[6] = {0, 0, 0, 0, 0, 0};
        bool has = false;
        const int64_t k = gk - tab.g_off[v];
        const bool in = valid && k >= 0 && k < tab.n[v];
        const int64_t r = in ? tab.r_off[v] + k : 0;
        const bool hit = ((hg >> v) & 1u) != 0u;
        float a[10];
        gather_adjoint(hit, r, M, copies, g2d, a);
        {
          if (hit) {
            has = true;
            touched[r] = 0;
            const gs_camera cam = cams[v];
            const ProjF P = project_f(cam, m, ls, q, op);
            gc[0] += a[6];
            gc[1] += a[7];
            gc[2] += a[8];
            if (P.kept) {
              const float k1 = P.k1, k2 = P.k2, k3 = P.k3;
              // conic -> 2D covariance
              const float G00 = a[2], G01 = 0.5f * a[3], G11 = a[4];
              const float QG00 = k1 * G00 + k2 * G01, QG01 = k1 * G01 + k2 * G11;
              const float QG10 = k2 * G00 + k3 * G01, QG11 = k2 * G01 + k3 * G11;
              const float cb00 = -(QG00 * k1 + QG01 * k2);
              const float cb01 = -(QG00 * k2 + QG01 * k3);
              const float cb11 = -(QG10 * k2 + QG11 * k3);
              // cov = JT JT^T + 0.3 I -> JTbar = 2 cb JT
              float JTb[2][3];
              for (int j = 0; j < 3; ++j) {
                JTb[0][j] = 2.f * (cb00 * P.JT[0][j] + cb01 * P.JT[1][j]);
                JTb[1][j] = 2.f * (cb01 * P.JT[0][j] + cb11 * P.JT[1][j]);
              }
              // JT = J T1
              const float Jb00 = JTb[0][0] * P.T1[0][0] + JTb[0][1] * P.T1[0][1] + JTb[0][2] * P.T1[0][2];
              const float Jb02 = JTb[0][0] * P.T1[2][0] + JTb[0][1] * P.T1[2][1] + JTb[0][2] * P.T1[2][2];
              const float Jb11 = JTb[1][0] * P.T1[1][0] + JTb[1][1] * P.T1[1][1] + JTb[1][2] * P.T1[1][2];
              const float Jb12 = JTb[1][0] * P.T1[2][0] + JTb[1][1] * P.T1[2][1] + JTb[1][2] * P.T1[2][2];
              float T1b[3][3];
              for (int j = 0; j < 3; ++j) {
                T1b[0][j] = P.j00 * JTb[0][j];
                T1b[1][j] = P.j11 * JTb[1][j];
                T1b[2][j] = P.j02 * JTb[0][j] + P.j12 * JTb[1][j];
              }
              const float x = P.px, y = P.py, iz = 1.0f / P.pz;
              const float iz2 = iz * iz, iz3 = iz2 * iz;
              const float fx = cam.fx, fy = cam.fy;
              float pb0 = Jb02 * (-fx * iz2) + a[0] * fx * iz;
              float pb1 = Jb12 * (-fy * iz2) + a[1] * fy * iz;
              float pb2 = Jb00 * (-fx * iz2) + Jb02 * (2.f * fx * x * iz3) + Jb11 * (-fy * iz2) +
                          Jb12 * (2.f * fy * y * iz3) - a[0] * fx * x * iz2 - a[1] * fy * y * iz2 + a[9];
              // pose: p' = Exp(xi) p and T1' = Exp(phi) T1
              float B[3][3];
              for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                  B[i][j] = P.T1[i][0] * T1b[j][0] + P.T1[i][1] * T1b[j][1] + P.T1[i][2] * T1b[j][2];
              pv[0] = pb0;
              pv[1] = pb1;
              pv[2] = pb2;
              pv[3] = y * pb2 - P.pz * pb1 + (B[1][2] - B[2][1]);
              pv[4] = P.pz * pb0 - x * pb2 + (B[2][0] - B[0][2]);
              pv[5] = x * pb1 - y * pb0 + (B[0][1] - B[1][0]);
              if (!pose_only) {
                const float* R = cam.T_cw;  // rows R[0..2], R[4..6], R[8..10]
                for (int c = 0; c < 3; ++c) gm[c] += R[c] * pb0 + R[4 + c] * pb1 + R[8 + c] * pb2;
                // T1 = R Mw, Mw = Rq diag(S): Mwbar = R^T T1bar
                float Mb[3][3];
                for (int i = 0; i < 3; ++i)
                  for (int j = 0; j < 3; ++j) Mb[i][j] = R[i] * T1b[0][j] + R[4 + i] * T1b[1][j] + R[8 + i] * T1b[2][j];
                float Rb[3][3];
                for (int j = 0; j < 3; ++j) {
                  const float sb = Mb[0][j] * P.Rq[0][j] + Mb[1][j] * P.Rq[1][j] + Mb[2][j] * P.Rq[2][j];
                  gl[j] += sb * P.S[j];
                  for (int i = 0; i < 3; ++i) Rb[i][j] = Mb[i][j] * P.S[j];
                }
                const float w = P.qn[0], qx = P.qn[1], qy = P.qn[2], qz = P.qn[3];
                float nb[4];
                nb[0] = 2.f * (-qz * Rb[0][1] + qy * Rb[0][2] + qz * Rb[1][0] - qx * Rb[1][2] - qy * Rb[2][0] +
                               qx * Rb[2][1]);
                nb[1] = 2.f * (qy * Rb[0][1] + qz * Rb[0][2] + qy * Rb[1][0] - 2.f * qx * Rb[1][1] - w * Rb[1][2] +
                               qz * Rb[2][0] + w * Rb[2][1] - 2.f * qx * Rb[2][2]);
                nb[2] = 2.f * (-2.f * qy * Rb[0][0] + qx * Rb[0][1] + w * Rb[0][2] + qx * Rb[1][0] + qz * Rb[1][2] -
                               w * Rb[2][0] + qz * Rb[2][1] - 2.f * qy * Rb[2][2]);
                nb[3] = 2.f * (-2.f * qz * Rb[0][0] - w * Rb[0][1] + qx * Rb[0][2] + w * Rb[1][0] -
                               2.f * qz * Rb[1][1] + qy * Rb[1][2] + qx * Rb[2][0] + qy * Rb[2][1]);
                const float dot = nb[0] * P.qn[0] + nb[1] * P.qn[1] + nb[2] * P.qn[2] + nb[3] * P.qn[3];
                for (int c = 0; c < 4; ++c) gq[c] += (nb[c] - P.qn[c] * dot) * P.qinv;
                go += a[5] * P.o * (1.f - P.o);
              }
            }
          }
        }
        if (__ballot(has) != 0) {
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const float x = wave_sum_to_lane63(pv[c]);
            if (lane == 63) s_pose[wv][v * 6 + c] += x;
          }
        }
      }
    }
    if (valid && !pose_only) {
      if (accumulate) {
        if (hg == 0u) continue;  // zero gradients leave the sums as they are
        for (int c = 0; c < 3; ++c) {
          d_mean[c * N + gk] += gm[c];
          d_ls[c * N + gk] += gl[c];
          d_color[c * N + gk] += gc[c];
        }
        for (int c = 0; c < 4; ++c) d_quat[c * N + gk] += gq[c];
        d_opl[gk] += go;
      } else {
        for (int c = 0; c < 3; ++c) {
          d_mean[c * N + gk] = gm[c];
          d_ls[c * N + gk] = gl[c];
          d_color[c * N + gk] = gc[c];
        }
        for (int c = 0; c < 4; ++c) d_quat[c * N + gk] = gq[c];
        d_opl[gk] = go;
      }
    }
  }
  // block partials [view][component][pstride]: the four wave sums in order
  __syncthreads();
  for (int i = threadIdx.x; i < tab.nv * 6; i += GS_BLOCK)
    pose_part[(int64_t)i * pstride + blockIdx.x] = s_pose[0][i] + s_pose[1][i] + s_pose[2][i] + s_pose[3][i];
}

// Sums one view's per-block pose partials in a fixed order (one workgroup per
// view, float64) and resets them to zero, so the scratch stays zero-filled.
// The partials are stored per component with a row stride that is a multiple
// of four, so each thread has 6 x kPoseGroup float4 loads in flight.
constexpr int kPoseGroup = 4;
__global__ __launch_bounds__(GS_BLOCK) void pose_final_kernel(float* __restrict__ part, int pstride,
                                                              float* __restrict__ pose, int accumulate) {
  __shared__ double s_red[GS_BLOCK / 64][6];
  const int v = blockIdx.x, lane = __lane_id(), w = threadIdx.x >> 6;
  float4* pv = reinterpret_cast<float4*>(part + (int64_t)v * 6 * pstride);
  const int n4 = pstride >> 2;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int j0 = threadIdx.x; j0 < n4; j0 += kPoseGroup * GS_BLOCK) {
    float4 x[6][kPoseGroup];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
#pragma unroll
      for (int u = 0; u < kPoseGroup; ++u) {
        const int j = j0 + u * GS_BLOCK;
        x[c][u] = j < n4 ? pv[c * n4 + j] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
#pragma unroll
      for (int u = 0; u < kPoseGroup; ++u) {
        acc[c] += (double)x[c][u].x;
        acc[c] += (double)x[c][u].y;
        acc[c] += (double)x[c][u].z;
        acc[c] += (double)x[c][u].w;
        const int j = j0 + u * GS_BLOCK;
        if (j < n4) pv[c * n4 + j] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }
  for (int c = 0; c < 6; ++c) {
    acc[c] = wave_sum_to_lane63_d(acc[c]);
    if (lane == 63) s_red[w][c] = acc[c];
  }
  __syncthreads();
  if (threadIdx.x < 6 && pose) {
    const int c = threadIdx.x;
    const double t = s_red[0][c] + s_red[1][c] + s_red[2][c] + s_red[3][c];
    pose[v * 6 + c] = (float)(accumulate ? (double)pose[v * 6 + c] + t : t);
  }
}

}  // namespace

gs_status launch_bwd_project(gs_ctx* ctx, const ViewTab& tab, const gs_camera* cams, const gs_gaussians* g,
                             float* g2d, uint8_t* touched, float* pose_part, gs_grads* gr, hipStream_t s) {
  const int nblk = bwd_pose_blocks(ctx, tab);
  {
    GS_LAUNCH(ctx, bwd_project_kernel, dim3(nblk), dim3(GS_BLOCK), 0, s, tab, cams, g->mean, g->log_scale,
                       g->quat, g->opacity_logit, g2d, touched, gr->mean, gr->log_scale, gr->quat, gr->opacity_logit,
                       gr->color, pose_part, bwd_pose_stride(ctx, tab), gr->pose_only, gr->accumulate,
                       ctx->bwd_copies);
  }
  GS_LAUNCH(ctx, pose_final_kernel, dim3(tab.nv), dim3(GS_BLOCK), 0, s, pose_part, bwd_pose_stride(ctx, tab), gr->pose,
            gr->accumulate);
  return gs_check_launch(ctx, "render_bwd_project");
}

// Blocks of bwd_project: one per group of GS_BLOCK Gaussians, at most as
// many as the device holds at once (queried once per context).
int bwd_pose_blocks(gs_ctx* ctx, const ViewTab& tab) {
  if (ctx->proj_resident <= 0) {
    int n = ctx->n_cu, per = 0;
    if (n <= 0 && (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess))
      n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)bwd_project_kernel, GS_BLOCK, 0) !=
        hipSuccess)
      per = 0;
    (void)hipGetLastError();
    ctx->proj_resident = n > 0 && per > 0 ? n * per : 1024;
  }
  const int64_t groups = (tab.ng + GS_BLOCK - 1) / GS_BLOCK;
  return (int)std::max<int64_t>(1, std::min<int64_t>(groups, ctx->proj_resident));
}

int bwd_pose_stride(gs_ctx* ctx, const ViewTab& tab) { return (bwd_pose_blocks(ctx, tab) + 3) & ~3; }
