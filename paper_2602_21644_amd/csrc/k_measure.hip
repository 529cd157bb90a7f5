// Measurement aid: float atomicAdd throughput on the access pattern of the
// backward's 2D-adjoint accumulation, the atomic roofline of that kernel.
//
// n_ops operations, in groups of ten consecutive floats (the ten adjoint
// components of one record): operation i adds 1 to component i % 10 of record
// r(i) = hash(i / 10) % n_records, in the accumulator copy of the XCD the
// workgroup runs on (copies 1, 2, 4 or 8, as the backward's "bwd_copies").
// Ten adjacent lanes serve one record, as in the backward's atomic pass.
#include "gs_internal.h"

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  // a fixed integer hash (xorshift-multiply), spreads consecutive groups
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(GS_BLOCK) void atomic_bench_kernel(float* __restrict__ acc, int64_t n_records,
                                                                int64_t n_ops, int copies) {
  float* base = acc;
  if (copies > 1)
    base += (int64_t)(__builtin_amdgcn_s_getreg((31 << 11) | 20) & (uint32_t)(copies - 1)) * 10 * n_records;
  for (int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x; i < n_ops; i += (int64_t)gridDim.x * GS_BLOCK) {
    const int64_t grp = i / 10, c = i - grp * 10;
    const int64_t r = (int64_t)(mix32((uint32_t)grp) % (uint32_t)n_records);
    atomicAdd(&base[r * 10 + c], 1.0f);
  }
}

}  // namespace

gs_status gs_measure_atomics(gs_ctx* ctx, float* acc, int64_t n_records, int64_t n_ops, int32_t copies,
                             void* stream) {
  if (!ctx || !acc || n_records < 1 || n_records > 0xFFFFFFFFLL || n_ops < 0) return gs_fail(ctx, GS_E_ARG, "bad argument");
  if (copies != 1 && copies != 2 && copies != 4 && copies != 8) return gs_fail(ctx, GS_E_ARG, "copies 1|2|4|8");
  if (n_ops == 0) return GS_OK;
  const int64_t blocks = std::min<int64_t>((n_ops + GS_BLOCK - 1) / GS_BLOCK, 8192);
  GS_LAUNCH(ctx, atomic_bench_kernel, dim3((unsigned)blocks), dim3(GS_BLOCK), 0, (hipStream_t)stream, acc,
            n_records, n_ops, copies);
  return gs_check_launch(ctx, "measure_atomics");
}
