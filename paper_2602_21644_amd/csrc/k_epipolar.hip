// Epipolar verification and static recovery near motion boundaries
// (Sec. IV-C, Eq. (18)-(19)).
//
// The fundamental matrix of the view pair, F = K2^-T [t]_x R K1^-1 with
// R = R2 R1^T and t = t2 - R t1, is formed in double from the two cameras in
// device memory (so it follows poses updated on the GPU); a relative
// translation shorter than 1e-6 leaves no baseline and F = 0.
//
// epi_select_kernel: one wave per candidate Gaussian. Its matches' distances
// d = |p2^T F p1| / |(a, b)|, (a, b, c) = F p1 (double, stored as float32 with
// NaN canonicalised to the positive quiet NaN), then the lower median of the
// segment over the float32 bit patterns (the distances are >= 0, so their bit
// patterns order like their values, NaN above +inf): a segment of at most 64
// matches holds one value per lane and finds the median by ranking every
// value against the others; a longer one by a radix select (8-bit digits,
// four passes, a 256-bin histogram per wave in LDS) that re-reads the
// distances the same lanes stored. Then the decision (mp > tau: suppressed;
// d_bar < eps: consistent) and the candidate's state. F is formed once per
// workgroup and shared through LDS.
//
// epi_restore_kernel: one thread per candidate writes mp_restore to the MP of
// every restored candidate. A pass of its own, so that every decision reads
// the MP from before the call even when a Gaussian is listed twice.
//
// HBM bound: 16 B read and 4 B written per match, about 25 B per candidate;
// the passes after the first re-read the distances from L2.
#include "gs_internal.h"

namespace {

constexpr uint32_t kQNaN = 0x7FC00000u;

struct Fund {
  double f[9];
};

__device__ Fund fundamental_of(const gs_camera& c1, const gs_camera& c2) {
  const float* A = c1.T_cw;
  const float* B = c2.T_cw;
  double R[3][3], t[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      R[i][j] = (double)B[4 * i] * A[4 * j] + (double)B[4 * i + 1] * A[4 * j + 1] + (double)B[4 * i + 2] * A[4 * j + 2];
  for (int i = 0; i < 3; ++i) t[i] = (double)B[4 * i + 3] - (R[i][0] * A[3] + R[i][1] * A[7] + R[i][2] * A[11]);
  Fund F;
  if (!(sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]) >= 1e-6)) {
    for (int i = 0; i < 9; ++i) F.f[i] = 0.0;
    return F;
  }
  // E = [t]_x R
  const double S[3][3] = {{0.0, -t[2], t[1]}, {t[2], 0.0, -t[0]}, {-t[1], t[0], 0.0}};
  double E[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) E[i][j] = S[i][0] * R[0][j] + S[i][1] * R[1][j] + S[i][2] * R[2][j];
  // K^-1 = [[1/fx, 0, -cx/fx], [0, 1/fy, -cy/fy], [0, 0, 1]]
  const double ia = 1.0 / c1.fx, ib = 1.0 / c1.fy, ic = -(double)c1.cx / c1.fx, id = -(double)c1.cy / c1.fy;
  const double ja = 1.0 / c2.fx, jb = 1.0 / c2.fy, jc = -(double)c2.cx / c2.fx, jd = -(double)c2.cy / c2.fy;
  // G = E K1^-1
  double G[3][3];
  for (int i = 0; i < 3; ++i) {
    G[i][0] = E[i][0] * ia;
    G[i][1] = E[i][1] * ib;
    G[i][2] = E[i][0] * ic + E[i][1] * id + E[i][2];
  }
  // F = K2^-T G, K2^-T = [[ja, 0, 0], [0, jb, 0], [jc, jd, 1]]
  for (int j = 0; j < 3; ++j) {
    F.f[j] = ja * G[0][j];
    F.f[3 + j] = jb * G[1][j];
    F.f[6 + j] = jc * G[0][j] + jd * G[1][j] + G[2][j];
  }
  return F;
}

__device__ __forceinline__ uint32_t epi_distance_bits(const Fund& F, float u1, float v1, float u2, float v2) {
  const double a = F.f[0] * u1 + F.f[1] * v1 + F.f[2];
  const double b = F.f[3] * u1 + F.f[4] * v1 + F.f[5];
  const double c = F.f[6] * u1 + F.f[7] * v1 + F.f[8];
  const double num = fabs((double)u2 * a + (double)v2 * b + c);
  const float d = (float)(num / sqrt(a * a + b * b));
  return d != d ? kQNaN : __float_as_uint(d);
}

// One wave's 256-bin histogram; waves of a workgroup run different segments,
// so only wave-level ordering is used (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The element of rank `rank` (bit-pattern order) of the distances of matches
// b .. e - 1, which this wave computes and stores to d in the first pass and
// reads back in the others (each lane the indices it stored). Radix select:
// four 8-bit digits from the top, a 256-bin histogram per pass.
__device__ uint32_t wave_radix_select(const Fund& F, const float* __restrict__ p1, const float* __restrict__ p2,
                                      int64_t m, int64_t b, int64_t e, uint32_t rank, float* __restrict__ d,
                                      uint32_t* hist, int lane) {
  uint32_t prefix = 0, mask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = lane; i < 256; i += 64) hist[i] = 0u;
    wave_lds_sync();
    for (int64_t i = b + lane; i < e; i += 64) {
      uint32_t x;
      if (shift == 24) {
        x = epi_distance_bits(F, p1[i], p1[m + i], p2[i], p2[m + i]);
        d[i] = __uint_as_float(x);
      } else {
        x = __float_as_uint(d[i]);
      }
      if ((x & mask) == prefix) atomicAdd(&hist[(x >> shift) & 255u], 1u);
    }
    wave_lds_sync();
    // lane L holds bins 4L .. 4L + 3; the digit is the first bin whose
    // running count passes the rank
    const uint32_t c0 = hist[4 * lane], c1 = hist[4 * lane + 1], c2 = hist[4 * lane + 2], c3 = hist[4 * lane + 3];
    const uint32_t s = c0 + c1 + c2 + c3;
    uint32_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += y;
    }
    const uint64_t hit = __ballot(incl > rank);
    const int L = __builtin_ctzll(hit);  // the counts sum to more than the rank, so some lane passes
    uint32_t acc = incl - s, dig = 0;
    if (acc + c0 > rank) {
      dig = 0;
    } else if (acc + c0 + c1 > rank) {
      dig = 1;
      acc += c0;
    } else if (acc + c0 + c1 + c2 > rank) {
      dig = 2;
      acc += c0 + c1;
    } else {
      dig = 3;
      acc += c0 + c1 + c2;
    }
    const uint32_t digit = 4u * (uint32_t)L + (uint32_t)__builtin_amdgcn_readlane((int)dig, L);
    rank -= (uint32_t)__builtin_amdgcn_readlane((int)acc, L);
    prefix |= digit << shift;
    mask |= 255u << shift;
  }
  return prefix;
}

__global__ __launch_bounds__(GS_BLOCK) void epi_select_kernel(
    const gs_camera* __restrict__ cams, int v1, int v2, const float* __restrict__ p1, const float* __restrict__ p2,
    int64_t m, const int32_t* __restrict__ ids, const int64_t* __restrict__ seg, int64_t K, int64_t n,
    const float* __restrict__ mp, float eps, float tau, float* __restrict__ d, float* __restrict__ dbar,
    uint8_t* __restrict__ state) {
  __shared__ uint32_t s_hist[GS_BLOCK / 64][256];
  __shared__ double s_F[9];
  // F once per workgroup (the only barrier: before any wave leaves)
  if (threadIdx.x == 0) {
    const Fund F0 = fundamental_of(cams[v1], cams[v2]);
    for (int i = 0; i < 9; ++i) s_F[i] = F0.f[i];
  }
  __syncthreads();
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * (GS_BLOCK / 64) + wv;
  if (k >= K) return;  // uniform per wave
  const int64_t id = ids[k], b = seg[k], e = seg[k + 1];
  if (id < 0 || id >= n || b < 0 || e < b || e > m || e - b >= ((int64_t)1 << 31)) {
    if (lane == 0) {
      dbar[k] = __uint_as_float(kQNaN);
      state[k] = 4;  // invalid
    }
    return;
  }
  if (e == b) {
    if (lane == 0) {
      dbar[k] = __uint_as_float(kQNaN);
      state[k] = 3;  // no matches
    }
    return;
  }
  Fund F;
  for (int i = 0; i < 9; ++i) F.f[i] = s_F[i];
  const float mpv = mp[id];
  const int64_t cnt = e - b;
  const uint32_t rank = (uint32_t)((cnt - 1) >> 1);  // lower median
  uint32_t med;
  if (cnt <= 64) {
    // one value per lane: its rank by comparison with every other (ties by
    // lane), and the lane whose rank is the median's
    const bool live = lane < cnt;
    uint32_t x = 0xFFFFFFFFu;
    if (live) {
      x = epi_distance_bits(F, p1[b + lane], p1[m + b + lane], p2[b + lane], p2[m + b + lane]);
      d[b + lane] = __uint_as_float(x);
    }
    uint32_t r = 0;
    for (int j = 0; j < (int)cnt; ++j) {
      const uint32_t y = (uint32_t)__builtin_amdgcn_readlane((int)x, j);
      r += (y < x || (y == x && j < lane)) ? 1u : 0u;
    }
    const uint64_t sel = __ballot(live && r == rank);
    med = (uint32_t)__builtin_amdgcn_readlane((int)x, __builtin_ctzll(sel));
  } else {
    med = wave_radix_select(F, p1, p2, m, b, e, rank, d, s_hist[wv], lane);
  }
  if (lane == 0) {
    const float md = __uint_as_float(med);
    dbar[k] = md;
    state[k] = !(mpv > tau) ? 2 : (md < eps ? 1 : 0);
  }
}

__global__ __launch_bounds__(GS_BLOCK) void epi_restore_kernel(const int32_t* __restrict__ ids,
                                                               const uint8_t* __restrict__ state, int64_t K,
                                                               float mp_restore, float* __restrict__ mp) {
  const int64_t k = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
  if (k < K && state[k] == 1) mp[ids[k]] = mp_restore;
}

}  // namespace

gs_status launch_epipolar(gs_ctx* ctx, const gs_camera* cams, int v1, int v2, const float* p1, const float* p2,
                          int64_t m, const int32_t* ids, const int64_t* seg, int64_t K, int64_t n, float eps,
                          float tau, float mp_restore, float* d, float* dbar, uint8_t* state, float* mp,
                          hipStream_t s) {
  if (K == 0) return GS_OK;
  const int64_t wpb = GS_BLOCK / 64;
  GS_LAUNCH(ctx, epi_select_kernel, dim3((unsigned)((K + wpb - 1) / wpb)), dim3(GS_BLOCK), 0, s, cams, v1, v2, p1,
            p2, m, ids, seg, K, n, mp, eps, tau, d, dbar, state);
  const gs_status st = gs_check_launch(ctx, "epipolar_select");
  if (st != GS_OK) return st;
  GS_LAUNCH(ctx, epi_restore_kernel, dim3((unsigned)((K + GS_BLOCK - 1) / GS_BLOCK)), dim3(GS_BLOCK), 0, s, ids,
            state, K, mp_restore, mp);
  return gs_check_launch(ctx, "epipolar_restore");
}
