// Second part of gs_render_bwd: per-Gaussian adjoint of the projection.
//
// The tile pass lists every Gaussian it gave a gradient (once per call) and
// clears the dense gradient outputs (each of its workgroups a slice, after
// its tile). kChainBlocks workgroups then walk the list, one thread per listed
// Gaussian: for every view of its scene it gathers the record's 2D adjoint
// (the sum of its per-XCD copies in a fixed order, every load in flight at
// once, the copies reset to zero so the scratch stays zero-filled), chains it
// through the projection in float32, sums the parameter gradients over the
// views in registers, stores them (or adds them when accumulating) and clears
// the Gaussian's flag; the pose-twist terms are summed per wave and per
// workgroup.
// The last workgroup with list entries to finish (a ticket counter with
// device-scope fences) sums the workgroups' pose partials in a fixed order
// and resets the list length and the ticket.
//
// The chain works with the camera-space square root T1 = R Rq diag(S) of the
// covariance (cov2D = (J T1)(J T1)^T + 0.3 I), a different route from the
// covariance-space derivation of the CPU reference.
#include "gs_project_dev.h"

namespace {

constexpr int kMaxCopies = 8;  // largest "bwd_copies"

__global__ __launch_bounds__(GS_BLOCK) void bwd_project_kernel(
    ViewTab tab, const gs_camera* __restrict__ cams, const float* __restrict__ mean,
    const float* __restrict__ log_scale, const float* __restrict__ quat, const float* __restrict__ opl,
    float* __restrict__ g2d, TouchArgs touch, float* __restrict__ d_mean, float* __restrict__ d_ls,
    float* __restrict__ d_quat, float* __restrict__ d_opl, float* __restrict__ d_color, float* __restrict__ pose_part,
    float* __restrict__ pose, int pose_only, int accumulate, int copies, int clear_all) {
  const int64_t N = tab.ng;
  const int64_t M = tab.nrec;
  if (clear_all) {
    // no tile pass ran (no tiles), so nothing is listed and no gradient was
    // cleared: every Gaussian gets zeros
    for (int64_t gk = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x; gk < N; gk += (int64_t)gridDim.x * GS_BLOCK) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        d_mean[c * N + gk] = 0.f;
        d_ls[c * N + gk] = 0.f;
        d_color[c * N + gk] = 0.f;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) d_quat[c * N + gk] = 0.f;
      d_opl[gk] = 0.f;
    }
  }
  __shared__ float s_pose[GS_BLOCK / 64][GS_MAX_VIEWS * 6];  // per-wave pose sums
  __shared__ uint32_t s_last;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int nvp = tab.nv * 6;
  // every workgroup reads the same length: the last working workgroup resets
  // it only after all working workgroups have taken their ticket
  const uint32_t cnt = *touch.count;
  const uint32_t nwork = min((cnt + GS_BLOCK - 1) / GS_BLOCK, (uint32_t)kChainBlocks);
  if (nwork == 0) {
    // nothing listed: the pose gradient is zero
    if (blockIdx.x == 0 && pose && !accumulate)
      for (int i = threadIdx.x; i < nvp; i += GS_BLOCK) pose[i] = 0.f;
    return;
  }
  if (blockIdx.x >= nwork) return;
  for (int i = lane; i < nvp; i += 64) s_pose[wv][i] = 0.f;
#pragma unroll 1
  for (uint32_t i0 = blockIdx.x * GS_BLOCK; i0 < cnt; i0 += kChainBlocks * GS_BLOCK) {  // uniform per block
    const uint32_t li = i0 + threadIdx.x;
    const bool valid = li < cnt;
    const int64_t gk = valid ? (int64_t)touch.list[li] : 0;
    if (valid) touch.list[li] = 0u;  // the scratch is left zero-filled
    float gm[3] = {0, 0, 0}, gl[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.f, gc[3] = {0, 0, 0};
    float m[3] = {0, 0, 0}, ls[3] = {0, 0, 0}, q[4] = {1, 0, 0, 0}, op = 0.f;
    if (valid) {
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
      const bool hit = valid && k >= 0 && k < tab.n[v];
      if (hit) {
        // the record's adjoint: its copies summed in a fixed order, then reset
        const int64_t r = tab.r_off[v] + k;
        float2 t[kMaxCopies][5];
#pragma unroll
        for (int cp = 0; cp < kMaxCopies; ++cp)
#pragma unroll
          for (int u = 0; u < 5; ++u)
            t[cp][u] = cp < copies ? reinterpret_cast<const float2*>(g2d + ((int64_t)cp * M + r) * 10)[u]
                                   : make_float2(0.f, 0.f);
        float a[10];
#pragma unroll
        for (int u = 0; u < 5; ++u) {
          float x = 0.f, y = 0.f;
#pragma unroll
          for (int cp = 0; cp < kMaxCopies; ++cp) {
            x += t[cp][u].x;
            y += t[cp][u].y;
          }
          a[2 * u] = x;
          a[2 * u + 1] = y;
        }
#pragma unroll
        for (int cp = 0; cp < kMaxCopies; ++cp)
          if (cp < copies)
#pragma unroll
            for (int u = 0; u < 5; ++u)
              reinterpret_cast<float2*>(g2d + ((int64_t)cp * M + r) * 10)[u] = make_float2(0.f, 0.f);
        {
            has = true;
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
    if (valid) {
      if (!pose_only) {
        if (accumulate) {
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
      touch.flag[gk] = 0u;
    }
  }
  // this workgroup's pose partials (the four wave sums in order), then a
  // ticket: the last working workgroup sums the partials in a fixed order.
  // Only the workgroups with list entries take part, and they store little,
  // so the device-scope fences stay cheap.
  __syncthreads();
  for (int i = threadIdx.x; i < nvp; i += GS_BLOCK)
    pose_part[(int64_t)blockIdx.x * nvp + i] = s_pose[0][i] + s_pose[1][i] + s_pose[2][i] + s_pose[3][i];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(touch.ticket, 1u) == nwork - 1u ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // wave w sums components w, w + 4, ...: each lane the partials of
  // workgroups lane, lane + 64, ... in double, then a fixed butterfly
  for (int i = wv; i < nvp; i += GS_BLOCK / 64) {
    double t = 0.0;
    for (uint32_t b = lane; b < nwork; b += 64) {
      t += (double)pose_part[(int64_t)b * nvp + i];
      pose_part[(int64_t)b * nvp + i] = 0.f;
    }
    t = wave_sum_all_d(t);
    if (lane == 0 && pose) pose[i] = (float)(accumulate ? (double)pose[i] + t : t);
  }
  if (threadIdx.x == 0) {
    *touch.count = 0u;
    *touch.ticket = 0u;
  }
}

}  // namespace

gs_status launch_bwd_project(gs_ctx* ctx, const ViewTab& tab, const gs_camera* cams, const gs_gaussians* g,
                             float* g2d, TouchArgs touch, float* pose_part, gs_grads* gr, hipStream_t s) {
  GS_LAUNCH(ctx, bwd_project_kernel, dim3(kChainBlocks), dim3(GS_BLOCK), 0, s, tab, cams, g->mean,
            g->log_scale, g->quat, g->opacity_logit, g2d, touch, gr->mean, gr->log_scale, gr->quat, gr->opacity_logit,
            gr->color, pose_part, gr->pose, gr->pose_only, gr->accumulate, ctx->bwd_copies,
            tab.ntiles == 0 && !gr->pose_only && !gr->accumulate ? 1 : 0);
  return gs_check_launch(ctx, "render_bwd_project");
}
