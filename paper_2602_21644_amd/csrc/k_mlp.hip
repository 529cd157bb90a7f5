// Learned per-pixel MP surrogate (not part of the paper): features, bfloat16
// weight sync, inference, and one Adam training step on the mean BCE.
//
// The net is 8 -> 32 -> 32 -> 1 (ReLU, ReLU, sigmoid): ~2.6 kFLOP per pixel,
// far too small a contraction for MFMA tiles to pay off at 64-pixel granularity
// against the VALU path; weights are expanded from bfloat16 into LDS once per
// workgroup and read as broadcasts, accumulation is float32.
#include "gs_internal.h"

namespace {

constexpr int NI = 8, NH = 32;
constexpr int OW1 = 0, OB1 = 256, OW2 = 288, OB2 = 1312, OW3 = 1344, OB3 = 1376, NP = 1377;
constexpr int QW1 = 0, QW2 = 256, QW3 = 1280, NQ = 1312;  // bfloat16 copy offsets
constexpr int SUB = 64;                                   // pixels per LDS sub-batch in training

__device__ __forceinline__ uint16_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Weights as used by the net, in LDS: W1, b1, W2, b2, W3, b3 (master layout).
__device__ __forceinline__ void load_net(float* s, const float* __restrict__ master, const uint16_t* __restrict__ wq) {
  for (int i = threadIdx.x; i < NP; i += blockDim.x) {
    float v;
    if (i < OB1) v = bf2f(wq[QW1 + i]);
    else if (i < OW2) v = master[i];
    else if (i < OB2) v = bf2f(wq[QW2 + (i - OW2)]);
    else if (i < OW3) v = master[i];
    else if (i < OB3) v = bf2f(wq[QW3 + (i - OW3)]);
    else v = master[i];
    s[i] = v;
  }
}

__device__ __forceinline__ float net_fwd(const float* s, const float x[NI], float z1[NH], float h1[NH], float z2[NH],
                                         float h2[NH]) {
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    float a = s[OB1 + i];
#pragma unroll
    for (int j = 0; j < NI; ++j) a = fmaf(s[OW1 + i * NI + j], x[j], a);
    z1[i] = a;
    h1[i] = fmaxf(a, 0.f);
  }
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    float a = s[OB2 + i];
#pragma unroll
    for (int j = 0; j < NH; ++j) a = fmaf(s[OW2 + i * NH + j], h1[j], a);
    z2[i] = a;
    h2[i] = fmaxf(a, 0.f);
  }
  float a = s[OB3];
#pragma unroll
  for (int j = 0; j < NH; ++j) a = fmaf(s[OW3 + j], h2[j], a);
  return a;
}

__global__ __launch_bounds__(GS_BLOCK) void mlp_features_kernel(int64_t P, int K, const float* __restrict__ C,
                                                                const float* __restrict__ D,
                                                                const float* __restrict__ Mm,
                                                                const float* __restrict__ T,
                                                                const float* __restrict__ Cg,
                                                                const float* __restrict__ Dg,
                                                                const int32_t* __restrict__ inst,
                                                                const float* __restrict__ prior,
                                                                float* __restrict__ x) {
  const int64_t p = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  if (p >= P) return;
  const float dg = Dg[p], d = D[p];
  x[p] = C[p] - Cg[p];
  x[P + p] = C[P + p] - Cg[P + p];
  x[2 * P + p] = C[2 * P + p] - Cg[2 * P + p];
  x[3 * P + p] = (dg > 0.f ? d - dg : 0.f) / 0.1f;
  x[4 * P + p] = Mm[p];
  x[5 * P + p] = T[p];
  x[6 * P + p] = d / 4.0f;
  x[7 * P + p] = prior[min(max(inst[p], 0), K)];
}

__global__ void mlp_sync_kernel(const float* __restrict__ master, uint16_t* __restrict__ wq) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NQ; i += gridDim.x * blockDim.x) {
    int src;
    if (i < QW2) src = OW1 + i;
    else if (i < QW3) src = OW2 + (i - QW2);
    else src = OW3 + (i - QW3);
    wq[i] = f2bf_rne(master[src]);
  }
}

__global__ __launch_bounds__(GS_BLOCK) void mlp_fwd_kernel(const float* __restrict__ master,
                                                           const uint16_t* __restrict__ wq,
                                                           const float* __restrict__ x, float* __restrict__ y,
                                                           int64_t P) {
  __shared__ float s[NP];
  load_net(s, master, wq);
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  if (p >= P) return;
  float xi[NI], z1[NH], h1[NH], z2[NH], h2[NH];
#pragma unroll
  for (int j = 0; j < NI; ++j) xi[j] = x[j * P + p];
  const float z3 = net_fwd(s, xi, z1, h1, z2, h2);
  y[p] = 1.f / (1.f + expf(-z3));
}

// Forward + backward per pixel; parameter gradients (of the mean BCE) summed
// per block in a fixed order and written as block partials.
__global__ __launch_bounds__(GS_BLOCK) void mlp_grad_kernel(const float* __restrict__ master,
                                                            const uint16_t* __restrict__ wq,
                                                            const float* __restrict__ x,
                                                            const float* __restrict__ label, int64_t P,
                                                            float* __restrict__ part, double* __restrict__ lpart) {
  __shared__ float s[NP];
  __shared__ float a_dz1[SUB][NH + 1], a_h1[SUB][NH + 1], a_dz2[SUB][NH + 1], a_h2[SUB][NH + 1], a_x[SUB][NI + 1];
  __shared__ float a_dz3[SUB];
  __shared__ double s_l[4];
  load_net(s, master, wq);
  __syncthreads();
  const float invP = 1.0f / (float)P;
  float acc[6] = {0, 0, 0, 0, 0, 0};
  double lsum = 0.0;
  const int64_t base = (int64_t)blockIdx.x * GS_BLOCK;
  for (int sb = 0; sb < GS_BLOCK / SUB; ++sb) {
    const int t = threadIdx.x;
    if (t < SUB) {
      const int64_t p = base + sb * SUB + t;
      if (p < P) {
        float xi[NI], z1[NH], h1[NH], z2[NH], h2[NH];
#pragma unroll
        for (int j = 0; j < NI; ++j) xi[j] = x[j * P + p];
        const float z3 = net_fwd(s, xi, z1, h1, z2, h2);
        const float yv = 1.f / (1.f + expf(-z3));
        const float tl = label[p];
        const float yc = fminf(fmaxf(yv, 1e-7f), 1.f - 1e-7f);
        lsum += -((double)tl * log((double)yc) + (1.0 - (double)tl) * log(1.0 - (double)yc));
        const float dz3 = (yv - tl) * invP;
        float dz2[NH];
#pragma unroll
        for (int i = 0; i < NH; ++i) dz2[i] = z2[i] > 0.f ? s[OW3 + i] * dz3 : 0.f;
#pragma unroll
        for (int j = 0; j < NH; ++j) {
          float a = 0.f;
#pragma unroll
          for (int i = 0; i < NH; ++i) a = fmaf(s[OW2 + i * NH + j], dz2[i], a);
          a_dz1[t][j] = z1[j] > 0.f ? a : 0.f;
          a_h1[t][j] = h1[j];
          a_dz2[t][j] = dz2[j];
          a_h2[t][j] = h2[j];
        }
#pragma unroll
        for (int j = 0; j < NI; ++j) a_x[t][j] = xi[j];
        a_dz3[t] = dz3;
      } else {
        for (int j = 0; j < NH; ++j) {
          a_dz1[t][j] = 0.f;
          a_h1[t][j] = 0.f;
          a_dz2[t][j] = 0.f;
          a_h2[t][j] = 0.f;
        }
        for (int j = 0; j < NI; ++j) a_x[t][j] = 0.f;
        a_dz3[t] = 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int idx = threadIdx.x + q * GS_BLOCK;
      if (idx >= NP) break;
      float a = 0.f;
      if (idx < OB1) {
        const int i = idx / NI, j = idx % NI;
        for (int p = 0; p < SUB; ++p) a = fmaf(a_dz1[p][i], a_x[p][j], a);
      } else if (idx < OW2) {
        const int i = idx - OB1;
        for (int p = 0; p < SUB; ++p) a += a_dz1[p][i];
      } else if (idx < OB2) {
        const int i = (idx - OW2) / NH, j = (idx - OW2) % NH;
        for (int p = 0; p < SUB; ++p) a = fmaf(a_dz2[p][i], a_h1[p][j], a);
      } else if (idx < OW3) {
        const int i = idx - OB2;
        for (int p = 0; p < SUB; ++p) a += a_dz2[p][i];
      } else if (idx < OB3) {
        const int j = idx - OW3;
        for (int p = 0; p < SUB; ++p) a = fmaf(a_dz3[p], a_h2[p][j], a);
      } else {
        for (int p = 0; p < SUB; ++p) a += a_dz3[p];
      }
      acc[q] += a;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int idx = threadIdx.x + q * GS_BLOCK;
    if (idx < NP) part[(int64_t)blockIdx.x * NP + idx] = acc[q];
  }
  lsum = wave_sum_all_d(lsum);
  if (__lane_id() == 63) s_l[threadIdx.x >> 6] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = s_l[0] + s_l[1] + s_l[2] + s_l[3];
}

__global__ __launch_bounds__(GS_BLOCK) void mlp_adam_kernel(const float* __restrict__ part,
                                                            const double* __restrict__ lpart, int nblk, int64_t P,
                                                            float lr, int step, float* __restrict__ master,
                                                            float* __restrict__ m, float* __restrict__ v,
                                                            float* __restrict__ grad_out, float* __restrict__ loss) {
  const int idx = blockIdx.x * GS_BLOCK + threadIdx.x;
  if (idx < NP) {
    double g = 0.0;
    for (int b = 0; b < nblk; ++b) g += (double)part[(int64_t)b * NP + idx];
    const float gf = (float)g;
    if (grad_out) grad_out[idx] = gf;
    const float b1 = 0.9f, b2 = 0.999f;
    const float mi = b1 * m[idx] + (1.f - b1) * gf;
    const float vi = b2 * v[idx] + (1.f - b2) * gf * gf;
    m[idx] = mi;
    v[idx] = vi;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    master[idx] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  }
  if (idx == 0) {
    double l = 0.0;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    *loss = (float)(l / (double)P);
  }
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t mlp_ws_bytes(int64_t P) {
  const int64_t nb = (P + GS_BLOCK - 1) / GS_BLOCK;
  return al((size_t)nb * NP * 4) + al((size_t)nb * 8);
}

gs_status launch_mlp_features(gs_ctx* ctx, const ViewTab& tab, const gs_image* img, const gs_target* tgt,
                              const gs_mp_frame* fr, float* x, hipStream_t s) {
  const int64_t P = tab.npix;
  if (P > 0)
    GS_LAUNCH(ctx, mlp_features_kernel, dim3((unsigned)((P + GS_BLOCK - 1) / GS_BLOCK)), dim3(GS_BLOCK), 0, s, P,
                       fr->n_inst, img->color, img->depth, img->mp, img->T, tgt->color, tgt->depth, fr->instance_id,
                       fr->inst_prior, x);
  return gs_check_launch(ctx, "mlp_features");
}

gs_status launch_mlp_sync(gs_ctx* ctx, gs_mlp* mlp, hipStream_t s) {
  GS_LAUNCH(ctx, mlp_sync_kernel, dim3(6), dim3(GS_BLOCK), 0, s, mlp->master, mlp->w_bf16);
  return gs_check_launch(ctx, "mlp_sync");
}

gs_status launch_mlp_fwd(gs_ctx* ctx, const gs_mlp* mlp, const float* x, float* y, int64_t P, hipStream_t s) {
  if (P > 0)
    GS_LAUNCH(ctx, mlp_fwd_kernel, dim3((unsigned)((P + GS_BLOCK - 1) / GS_BLOCK)), dim3(GS_BLOCK), 0, s,
                       mlp->master, mlp->w_bf16, x, y, P);
  return gs_check_launch(ctx, "mlp_fwd");
}

gs_status launch_mlp_train(gs_ctx* ctx, gs_mlp* mlp, const float* x, const float* label, int64_t P, float lr,
                           int step, float* loss, float* grad, char* ws, hipStream_t s) {
  const int nb = (int)((P + GS_BLOCK - 1) / GS_BLOCK);
  float* part = (float*)ws;
  double* lpart = (double*)(ws + al((size_t)nb * NP * 4));
  GS_LAUNCH(ctx, mlp_grad_kernel, dim3(nb), dim3(GS_BLOCK), 0, s, mlp->master, mlp->w_bf16, x, label, P, part,
                     lpart);
  GS_LAUNCH(ctx, mlp_adam_kernel, dim3((NP + GS_BLOCK - 1) / GS_BLOCK), dim3(GS_BLOCK), 0, s, part, lpart, nb, P,
                     lr, step, mlp->master, mlp->adam_m, mlp->adam_v, grad, loss);
  GS_LAUNCH(ctx, mlp_sync_kernel, dim3(6), dim3(GS_BLOCK), 0, s, mlp->master, mlp->w_bf16);
  return gs_check_launch(ctx, "mlp_train_step");
}
