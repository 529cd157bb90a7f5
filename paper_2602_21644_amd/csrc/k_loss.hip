// gs_loss: MP-weighted L1 colour + depth loss and its per-pixel adjoints.
// One thread per pixel; per-view loss summed in float64, per block, then in a
// fixed order by a one-workgroup kernel, so the value is run-to-run identical.
#include "gs_internal.h"

namespace {

__global__ __launch_bounds__(GS_BLOCK) void loss_kernel(ViewTab tab, const float* __restrict__ C,
                                                        const float* __restrict__ D, const float* __restrict__ Mm,
                                                        const float* __restrict__ T, LossArgs la) {
  __shared__ double s[4];
  const int v = blockIdx.y;
  const int64_t npx = (int64_t)tab.W[v] * tab.H[v];
  const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  const int64_t P = tab.npix;
  double acc = 0.0;
  if (i < npx) {
    const int64_t p = tab.px_off[v] + i;
    acc = pixel_loss(la, P, p, C[p], C[P + p], C[2 * P + p], D[p], Mm[p], T[p], la.Cg[p], la.Cg[P + p],
                     la.Cg[2 * P + p], la.Dg[p]);
  }
  acc = wave_sum_all_d(acc);
  if (__lane_id() == 63) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) la.part[(int64_t)v * gridDim.x + blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// Sums the per-block partials of a view in a fixed order (one workgroup per
// view); each thread has eight loads in flight before it sums them.
constexpr int kLossUnroll = 8;
__global__ __launch_bounds__(GS_BLOCK) void loss_final_kernel(const double* __restrict__ part, int nblk,
                                                              float* __restrict__ loss) {
  __shared__ double s[GS_BLOCK / 64];
  const int v = blockIdx.x;
  const double* pv = part + (int64_t)v * nblk;
  double t = 0.0;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += kLossUnroll * GS_BLOCK) {
    double x[kLossUnroll];
#pragma unroll
    for (int u = 0; u < kLossUnroll; ++u) x[u] = b0 + u * GS_BLOCK < nblk ? pv[b0 + u * GS_BLOCK] : 0.0;
#pragma unroll
    for (int u = 0; u < kLossUnroll; ++u) t += x[u];
  }
  t = wave_sum_all_d(t);
  if (__lane_id() == 63) s[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) loss[v] = (float)(s[0] + s[1] + s[2] + s[3]);
}

}  // namespace

LossArgs loss_args(const gs_target* tgt, const gs_loss_params* lp, gs_pixel_grads* pg, double* part, float* loss) {
  LossArgs la;
  la.Cg = tgt->color;
  la.Dg = tgt->depth;
  la.lp = lp->lambda_pho;
  la.ld = lp->lambda_depth;
  la.epsA = lp->eps_A;
  la.wmode = lp->weight_mode;
  la.gtw = lp->grad_through_weight;
  la.dC = pg->dcolor;
  la.dD = pg->ddepth;
  la.dM = pg->dmp;
  la.dT = pg->dT;
  la.part = part;
  la.loss = loss;
  return la;
}

int loss_blocks(const ViewTab& tab) {
  int64_t mx = 0;
  for (int v = 0; v < tab.nv; ++v) mx = (int64_t)tab.W[v] * tab.H[v] > mx ? (int64_t)tab.W[v] * tab.H[v] : mx;
  return (int)((mx + GS_BLOCK - 1) / GS_BLOCK);
}

gs_status launch_loss(gs_ctx* ctx, const ViewTab& tab, const gs_image* img, const gs_target* tgt,
                      const gs_loss_params* lp, float* loss, gs_pixel_grads* pg, double* part, hipStream_t s) {
  const int nb = loss_blocks(tab);
  if (nb == 0) return GS_OK;
  GS_LAUNCH(ctx, loss_kernel, dim3(nb, tab.nv), dim3(GS_BLOCK), 0, s, tab, img->color, img->depth, img->mp,
            img->T, loss_args(tgt, lp, pg, part, loss));
  GS_LAUNCH(ctx, loss_final_kernel, dim3(tab.nv), dim3(GS_BLOCK), 0, s, part, nb, loss);
  return gs_check_launch(ctx, "loss");
}
