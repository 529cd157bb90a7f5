// Prefix path of gs_bin_sort (bins->max_rank > 0 and a key histogram from
// gs_project).
//
// Compositing stops once a pixel's transmittance drops below 1e-4, so only a
// short front part of every tile list is ever read. This path bins exactly
// the records in front of a depth threshold: theta is the first boundary of
// the 4096-bin histogram of (depth key >> 20) at which at least max_rank
// records lie in front. Every tile list is then the exact prefix of its full
// list (all entries with key < theta, in the same order). If a tile runs out
// of its prefix with light still passing, gs_render_fwd raises `incomplete`
// and the caller re-bins with the full path.
//
// Kernels: select+count -> stable compaction -> one-workgroup LSD radix sort of
// the selection (+ instance prefix and chunk boundaries) -> per-chunk tile
// counts -> two-kernel segmented scan -> LDS-staged scatter. Chunks hold at
// most `budget` instances, so a chunk's part of every tile list is assembled in
// LDS and written out contiguously.
#include "bin_common.h"
#include "gs_project_dev.h"

namespace {

constexpr int HB = 4096;                        // coarse histogram bins
constexpr int SEL_ITEMS = 8;
constexpr int SEL_TILE = GS_BLOCK * SEL_ITEMS;  // records per select/compact block
constexpr int SORT_THREADS = 1024;
constexpr int SORT_WAVES = SORT_THREADS / 64;
constexpr int SCAN_TILE2 = 4096;

__device__ __forceinline__ int sel_blocks(int64_t npad) { return (int)((npad + SEL_TILE - 1) / SEL_TILE); }

// Threshold from the coarse histogram of one view: keys < theta are selected.
__device__ uint32_t theta_of(const uint32_t* __restrict__ hist, int64_t R, uint32_t* s_wave) {
  __shared__ uint32_t s_theta;
  constexpr int PER = HB / GS_BLOCK;
  uint32_t loc[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    loc[i] = hist[threadIdx.x * PER + i];
    sum += loc[i];
  }
  uint32_t total;
  const uint32_t ex = block_excl_scan(sum, s_wave, total);
  if (threadIdx.x == 0) s_theta = 0xFFFFFFFFu;
  __syncthreads();
  if ((int64_t)total > R) {
    uint32_t run = ex;
    for (int i = 0; i < PER; ++i) {
      const uint32_t nxt = run + loc[i];
      if ((int64_t)run < R && (int64_t)nxt >= R) s_theta = (uint32_t)(threadIdx.x * PER + i + 1) << 20;
      run = nxt;
    }
  }
  __syncthreads();
  return s_theta;
}

__global__ __launch_bounds__(GS_BLOCK) void sel_count_kernel(ViewTab tab, const uint32_t* __restrict__ key,
                                                             const uint32_t* __restrict__ hist, int64_t R,
                                                             int nb_max, uint32_t* __restrict__ theta_out,
                                                             uint32_t* __restrict__ cnt,
                                                             int32_t* __restrict__ overflow) {
  __shared__ uint32_t s_wave[4];
  const int v = blockIdx.y, b = blockIdx.x;
  if (v == 0 && b == 0 && threadIdx.x == 0) *overflow = 0;
  const int64_t npad = tab.npad[v];
  if (b >= sel_blocks(npad)) return;
  const uint32_t theta = theta_of(hist + (int64_t)v * HB, R, s_wave);
  if (b == 0 && threadIdx.x == 0) theta_out[v] = theta;
  uint32_t c = 0;
  const uint32_t* kv = key + tab.r_off[v];
#pragma unroll
  for (int i = 0; i < SEL_ITEMS; ++i) {
    const int64_t j = (int64_t)b * SEL_TILE + i * GS_BLOCK + threadIdx.x;
    if (j < npad) {
      const uint32_t k = kv[j];
      c += (k != 0xFFFFFFFFu && k < theta) ? 1u : 0u;
    }
  }
  uint32_t tot;
  block_excl_scan(c, s_wave, tot);
  if (threadIdx.x == 0) cnt[(int64_t)v * nb_max + b] = tot;
}

__global__ __launch_bounds__(GS_BLOCK) void compact_kernel(ViewTab tab, const uint32_t* __restrict__ key,
                                                           const uint32_t* __restrict__ theta_in,
                                                           const uint32_t* __restrict__ cnt, int nb_max,
                                                           uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ ckey, uint32_t* __restrict__ cid,
                                                           uint32_t* __restrict__ nsel) {
  __shared__ uint32_t s_wave[4];
  const int v = blockIdx.y, b = blockIdx.x;
  const int64_t npad = tab.npad[v];
  const int nb = sel_blocks(npad);
  if (b >= nb) return;
  const uint32_t theta = theta_in[v];
  uint32_t pre = 0;
  for (int i = threadIdx.x; i < b; i += GS_BLOCK) pre += cnt[(int64_t)v * nb_max + i];
  uint32_t tot;
  block_excl_scan(pre, s_wave, tot);
  uint32_t run = tot;  // records selected by earlier blocks
  const int64_t roff = tab.r_off[v];
  for (int i = 0; i < SEL_ITEMS; ++i) {
    const int64_t j = (int64_t)b * SEL_TILE + i * GS_BLOCK + threadIdx.x;
    uint32_t k = 0xFFFFFFFFu;
    if (j < npad) k = key[roff + j];
    const bool s = k != 0xFFFFFFFFu && k < theta;
    uint32_t t2;
    const uint32_t ex = block_excl_scan(s ? 1u : 0u, s_wave, t2);
    if (s) {
      ckey[roff + run + ex] = k;
      cid[roff + run + ex] = (uint32_t)j;
    }
    run += t2;
  }
  if (b == nb - 1 && threadIdx.x == 0) nsel[v] = run;
  // the histogram is consumed: clear it for the next projection
  for (int i = b * GS_BLOCK + threadIdx.x; i < HB; i += nb * GS_BLOCK) hist[(int64_t)v * HB + i] = 0;
}

// Inclusive scan over a 1024-thread block (16 waves).
__device__ __forceinline__ uint32_t block1024_excl(uint32_t x, uint32_t* s_w /*[16]*/, uint32_t& total) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int i = 0; i < SORT_WAVES; ++i) {
    const uint32_t t = s_w[i];
    if (i < w) base += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + inc - x;
}

// One workgroup per view: stable LSD radix sort of the selected (key, id)
// pairs on (key - min key), only over the digits the key range needs; then
// the instance count prefix in sorted order and the chunk boundaries.
__global__ __launch_bounds__(SORT_THREADS) void sel_sort_kernel(
    ViewTab tab, uint32_t* __restrict__ ka, uint32_t* __restrict__ ia, uint32_t* __restrict__ kb,
    uint32_t* __restrict__ ib, const uint32_t* __restrict__ nsel, const int2* __restrict__ rect,
    uint32_t* __restrict__ sorted_ids, int budget, int maxchunk, uint32_t* __restrict__ chunk_begin,
    uint32_t* __restrict__ nchunk_out, int64_t capacity, int32_t* __restrict__ overflow) {
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_wcnt[SORT_WAVES][256];
  __shared__ uint32_t s_w[SORT_WAVES];
  __shared__ uint32_t s_min, s_max;
  __shared__ uint32_t s_ex[SORT_THREADS];
  __shared__ uint32_t s_last_ex;
  __shared__ uint32_t s_maxb;
  const int v = blockIdx.x;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const uint32_t n = nsel[v];
  const int64_t roff = tab.r_off[v];
  if (threadIdx.x == 0) {
    s_min = 0xFFFFFFFFu;
    s_max = 0u;
  }
  __syncthreads();
  uint32_t lmin = 0xFFFFFFFFu, lmax = 0u;
  for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) {
    const uint32_t k = ka[roff + i];
    lmin = min(lmin, k);
    lmax = max(lmax, k);
  }
  atomicMin(&s_min, lmin);
  atomicMax(&s_max, lmax);
  __syncthreads();
  const uint32_t kmin = s_min;
  const uint32_t range = n > 0 ? s_max - kmin : 0u;
  const int bits = range ? 32 - __clz(range) : 0;
  int passes = (bits + 7) >> 3;
  uint32_t *sk = ka, *si = ia, *dk = kb, *di = ib;
  const uint64_t lt = lanemask_lt();
  // Fast path: one counting pass on the top 12 bits of (key - kmin) into 4096
  // buckets (order inside a bucket arbitrary), then each bucket sorted on
  // (key, id) by insertion. Taken when no bucket holds more than 64 records;
  // otherwise the stable LSD passes below run on the compacted input.
  {
    uint32_t* cur = &s_wcnt[0][0];  // 4096 bucket cursors
    const int sh = bits > 12 ? bits - 12 : 0;
    for (int i = threadIdx.x; i < 4096; i += SORT_THREADS) cur[i] = 0;
    if (threadIdx.x == 0) s_maxb = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) atomicAdd(&cur[(ka[roff + i] - kmin) >> sh], 1u);
    __syncthreads();
    uint32_t c4[4], s4 = 0, m4 = 0;
    for (int q = 0; q < 4; ++q) {
      c4[q] = cur[threadIdx.x * 4 + q];
      s4 += c4[q];
      m4 = max(m4, c4[q]);
    }
    atomicMax(&s_maxb, m4);
    uint32_t tot;
    uint32_t run = block1024_excl(s4, s_w, tot);
    for (int q = 0; q < 4; ++q) {
      cur[threadIdx.x * 4 + q] = run;
      run += c4[q];
    }
    __syncthreads();
    if (s_maxb <= 64) {
      for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS) {
        const uint32_t k = ka[roff + i];
        const uint32_t pos = atomicAdd(&cur[(k - kmin) >> sh], 1u);
        kb[roff + pos] = k;
        ib[roff + pos] = ia[roff + i];
      }
      __syncthreads();
      for (int q = 0; q < 4; ++q) {
        const int d = threadIdx.x * 4 + q;
        const uint32_t b0 = d ? cur[d - 1] : 0u, b1 = cur[d];
        for (uint32_t i = b0 + 1; i < b1; ++i) {
          const uint32_t k = kb[roff + i], id = ib[roff + i];
          uint32_t j = i;
          while (j > b0) {
            const uint32_t pk = kb[roff + j - 1], pid = ib[roff + j - 1];
            if (pk < k || (pk == k && pid < id)) break;
            kb[roff + j] = pk;
            ib[roff + j] = pid;
            --j;
          }
          kb[roff + j] = k;
          ib[roff + j] = id;
        }
      }
      __syncthreads();
      sk = kb;
      si = ib;
      passes = 0;
    }
  }
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * 8;
    if (threadIdx.x < 256) s_hist[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < SORT_WAVES * 256; i += SORT_THREADS) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += SORT_THREADS)
      atomicAdd(&s_hist[((sk[roff + i] - kmin) >> shift) & 255u], 1u);
    __syncthreads();
    if (threadIdx.x < 64) {
      // exclusive scan of 256 digit counts by one wave (4 per lane)
      uint32_t c[4], s = 0;
      for (int q = 0; q < 4; ++q) {
        c[q] = s_hist[lane * 4 + q];
        s += c[q];
      }
      uint32_t inc = s;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      uint32_t run = inc - s;
      for (int q = 0; q < 4; ++q) {
        s_base[lane * 4 + q] = run;
        run += c[q];
      }
    }
    __syncthreads();
    for (uint32_t r0 = 0; r0 < n; r0 += SORT_THREADS) {
      const uint32_t j = r0 + threadIdx.x;
      const bool valid = j < n;
      const uint32_t k = valid ? sk[roff + j] : 0u;
      const uint32_t id = valid ? si[roff + j] : 0u;
      const uint32_t d = ((k - kmin) >> shift) & 255u;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t m = __ballot(on);
        peers &= on ? m : ~m;
      }
      const uint32_t rank = __popcll(peers & lt);
      if (valid && rank == 0) s_wcnt[w][d] = __popcll(peers);
      __syncthreads();
      if (threadIdx.x < 256) {
        uint32_t o = s_base[threadIdx.x];
        for (int q = 0; q < SORT_WAVES; ++q) {
          const uint32_t c = s_wcnt[q][threadIdx.x];
          s_wcnt[q][threadIdx.x] = o;
          o += c;
        }
        s_base[threadIdx.x] = o;
      }
      __syncthreads();
      if (valid) {
        const uint32_t pos = s_wcnt[w][d] + rank;
        dk[roff + pos] = k;
        di[roff + pos] = id;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < SORT_WAVES * 256; i += SORT_THREADS) (&s_wcnt[0][0])[i] = 0;
      __syncthreads();
    }
    uint32_t* t;
    t = sk; sk = dk; dk = t;
    t = si; si = di; di = t;
  }
  // sorted ids, instance prefix and chunk boundaries
  uint32_t carry = 0, prev_ex = 0;
  uint32_t* cb = chunk_begin + (int64_t)v * (maxchunk + 1);
  for (uint32_t r0 = 0; r0 < n; r0 += SORT_THREADS) {
    const uint32_t j = r0 + threadIdx.x;
    const bool valid = j < n;
    uint32_t nt = 0;
    if (valid) {
      const uint32_t id = si[roff + j];
      sorted_ids[roff + j] = id;
      int x0, y0, x1, y1;
      rect_of(rect[roff + id], x0, y0, x1, y1);
      nt = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
    }
    uint32_t tot;
    const uint32_t ex = carry + block1024_excl(nt, s_w, tot);
    s_ex[threadIdx.x] = ex;
    __syncthreads();
    if (valid) {
      if (j == n - 1) s_last_ex = ex;
      const uint32_t before = threadIdx.x > 0 ? s_ex[threadIdx.x - 1] : prev_ex;
      const uint32_t c = ex / (uint32_t)budget;
      if ((j == 0 || before / (uint32_t)budget != c) && c < (uint32_t)maxchunk) cb[c] = j;
    }
    __syncthreads();
    prev_ex = s_ex[SORT_THREADS - 1];
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // chunk ids follow the records' exclusive instance prefix; every record
    // has 1 .. T instances and budget > T, so ids 0 .. last are all used
    uint32_t nc = 1;
    if (n > 0) nc = s_last_ex / (uint32_t)budget + 1;
    else cb[0] = 0;
    if (nc > (uint32_t)maxchunk) {
      nc = (uint32_t)maxchunk;
      *overflow = 1;
    }
    if ((int64_t)carry > capacity) *overflow = 1;
    cb[nc] = n;
    nchunk_out[v] = nc;
  }
}

struct PrefTab {
  int maxchunk;                  // chunk capacity per view (grid, strides)
  int budget;                    // instances per chunk before the last record
  int nbs[GS_MAX_VIEWS];         // scan blocks of the view's count matrix (host bound)
  int64_t cm_off[GS_MAX_VIEWS];  // view offset in the count matrix
  int64_t part_off[GS_MAX_VIEWS];
};

__device__ __forceinline__ int chunk_of(int b, int nchunk) {
  const int per = (nchunk + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__global__ __launch_bounds__(GS_BLOCK) void pcount_kernel(ViewTab tab, PrefTab pt,
                                                          const uint32_t* __restrict__ chunk_begin,
                                                          const uint32_t* __restrict__ nchunk_in,
                                                          const uint32_t* __restrict__ sorted,
                                                          const int2* __restrict__ rect,
                                                          uint32_t* __restrict__ cm,
                                                          const gs_camera* __restrict__ cams, GaussSrc gsrc,
                                                          float4* __restrict__ rec) {
  extern __shared__ int s_diff[];
  const int v = blockIdx.y;
  const int nchunk = (int)nchunk_in[v];
  const int c = chunk_of(blockIdx.x, nchunk);
  if (blockIdx.x >= (unsigned)(((nchunk + 7) >> 3) << 3) || c >= nchunk) return;
  const int gx = tab.gx[v], gy = tab.gy[v];
  const int cells = (gx + 1) * (gy + 1);
  for (int i = threadIdx.x; i < cells; i += GS_BLOCK) s_diff[i] = 0;
  __syncthreads();
  const uint32_t* cb = chunk_begin + (int64_t)v * (pt.maxchunk + 1);
  const uint32_t r0 = cb[c], r1 = cb[c + 1];
  const int64_t roff = tab.r_off[v];
  const gs_camera cam = cams[v];
  for (uint32_t i = r0 + threadIdx.x; i < r1; i += GS_BLOCK) {
    const uint32_t id = sorted[roff + i];
    int x0, y0, x1, y1;
    rect_of(rect[roff + id], x0, y0, x1, y1);
    diff_add(s_diff, gx + 1, x0, y0, x1, y1);
    // the compositing record of every selected record is written here once
    float4 a, b, cc;
    render_record(cam, gsrc, tab.g_off[v] + id, a, b, cc);
    rec[3 * (roff + id) + 0] = a;
    rec[3 * (roff + id) + 1] = b;
    rec[3 * (roff + id) + 2] = cc;
  }
  __syncthreads();
  diff_integrate(s_diff, gx, gy, threadIdx.x >> 6, GS_BLOCK / 64);
  const int T = gx * gy;
  uint32_t* out = cm + pt.cm_off[v] + c;
  for (int t = threadIdx.x; t < T; t += GS_BLOCK) {
    const int ty = t / gx, tx = t - ty * gx;
    out[(int64_t)t * nchunk] = (uint32_t)s_diff[ty * (gx + 1) + tx];
  }
}

// Segmented scan over each view's T x nchunk count matrix (device length).
__global__ __launch_bounds__(GS_BLOCK) void pscan_reduce_kernel(ViewTab tab, PrefTab pt,
                                                                const uint32_t* __restrict__ nchunk_in,
                                                                const uint32_t* __restrict__ cm,
                                                                uint32_t* __restrict__ part) {
  __shared__ uint32_t s_wave[4];
  const int v = blockIdx.y, b = blockIdx.x;
  if (b >= pt.nbs[v]) return;
  const int64_t len = (int64_t)tab.gx[v] * tab.gy[v] * nchunk_in[v];
  const int64_t base = (int64_t)b * SCAN_TILE2;
  uint32_t sum = 0;
  for (int i = threadIdx.x; i < SCAN_TILE2; i += GS_BLOCK) {
    const int64_t j = base + i;
    if (j < len) sum += cm[pt.cm_off[v] + j];
  }
  uint32_t tot;
  block_excl_scan(sum, s_wave, tot);
  if (threadIdx.x == 0) part[pt.part_off[v] + b] = tot;
}

__global__ __launch_bounds__(GS_BLOCK) void pscan_apply_kernel(ViewTab tab, PrefTab pt,
                                                               const uint32_t* __restrict__ nchunk_in,
                                                               uint32_t* __restrict__ cm,
                                                               const uint32_t* __restrict__ part,
                                                               int64_t total_parts, int64_t capacity,
                                                               uint32_t* __restrict__ tile_start,
                                                               int64_t* __restrict__ n_inst,
                                                               int32_t* __restrict__ overflow,
                                                               int32_t* __restrict__ incomplete) {
  __shared__ uint32_t s_wave[4];
  const int v = blockIdx.y, b = blockIdx.x;
  if (b >= pt.nbs[v]) return;
  // prefix: all partials of earlier views and of earlier blocks of this view
  const int64_t lim = pt.part_off[v] + b;
  uint64_t pre = 0;
  for (int64_t i = threadIdx.x; i < lim; i += GS_BLOCK) pre += part[i];
  uint32_t tot;
  const uint32_t pre32 = (uint32_t)pre;
  block_excl_scan(pre32, s_wave, tot);
  const uint32_t prefix = tot;
  if (v == 0 && b == 0) {
    uint64_t all = 0;
    for (int64_t i = threadIdx.x; i < total_parts; i += GS_BLOCK) all += part[i];
    uint32_t t2;
    block_excl_scan((uint32_t)all, s_wave, t2);
    if (threadIdx.x == 0) {
      tile_start[tab.ntiles] = t2;
      *n_inst = t2;
      *overflow = ((int64_t)t2 > capacity || *overflow) ? 1 : 0;
      if (incomplete) *incomplete = 0;
    }
  }
  const int nchunk = (int)nchunk_in[v];
  const int64_t len = (int64_t)tab.gx[v] * tab.gy[v] * nchunk;
  const int64_t base = (int64_t)b * SCAN_TILE2;
  constexpr int PER = SCAN_TILE2 / GS_BLOCK;
  uint32_t vals[PER];
  uint32_t sum = 0;
  const int64_t my = base + (int64_t)threadIdx.x * PER;
  uint32_t* a = cm + pt.cm_off[v];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    vals[i] = (my + i < len) ? a[my + i] : 0u;
    sum += vals[i];
  }
  uint32_t t3;
  uint32_t run = block_excl_scan(sum, s_wave, t3) + prefix;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int64_t e = my + i;
    if (e < len) {
      a[e] = run;
      if (e % nchunk == 0) tile_start[tab.tile_base[v] + e / nchunk] = run;
    }
    run += vals[i];
  }
}

// LDS-staged scatter of one chunk: the chunk's entries of every tile are
// placed in LDS in (tile, record) order, then copied out so each tile's run
// of entries is one contiguous write.
__global__ __launch_bounds__(GS_BLOCK) void pscatter_kernel(ViewTab tab, PrefTab pt,
                                                            const uint32_t* __restrict__ chunk_begin,
                                                            const uint32_t* __restrict__ nchunk_in,
                                                            const uint32_t* __restrict__ sorted,
                                                            const int2* __restrict__ rect,
                                                            const uint32_t* __restrict__ cm,
                                                            const int64_t* __restrict__ n_inst,
                                                            const int32_t* __restrict__ overflow,
                                                            uint32_t* __restrict__ out_ids, int maxT, int maxcells,
                                                            int cap_entries, int nw) {
  extern __shared__ int s_mem[];
  if (*overflow) return;
  const int v = blockIdx.y;
  const int nchunk = (int)nchunk_in[v];
  const int c = chunk_of(blockIdx.x, nchunk);
  if (blockIdx.x >= (unsigned)(((nchunk + 7) >> 3) << 3) || c >= nchunk) return;
  const int gx = tab.gx[v], gy = tab.gy[v];
  const int stride = gx + 1;
  const int cells = stride * (gy + 1);
  const int T = gx * gy;
  int* wd = s_mem;                                   // [nw][maxcells]
  int* lo = wd + nw * maxcells;                      // [maxT]
  uint32_t* gst = (uint32_t*)(lo + maxT);            // [maxT]
  uint32_t* ent = gst + maxT;                        // [cap_entries]
  uint16_t* etile = (uint16_t*)(ent + cap_entries);  // [cap_entries]
  __shared__ uint32_t s_wave[4];
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < nw * cells; i += GS_BLOCK) {
    const int ww = i / cells, cc = i - ww * cells;
    wd[ww * maxcells + cc] = 0;
  }
  __syncthreads();
  const uint32_t* cb = chunk_begin + (int64_t)v * (pt.maxchunk + 1);
  const uint32_t r0 = cb[c], r1 = cb[c + 1];
  // the first nw waves place the chunk's records, in nw consecutive ranges
  const uint32_t q = (r1 - r0 + nw - 1) / nw;
  const uint32_t wlo = w < nw ? min(r1, r0 + w * q) : r1, whi = w < nw ? min(r1, r0 + (w + 1) * q) : r1;
  const int64_t roff = tab.r_off[v];
  int* my = wd + (w < nw ? w : 0) * maxcells;
  for (uint32_t i = wlo + lane; i < whi; i += 64) {
    int x0, y0, x1, y1;
    rect_of(rect[roff + sorted[roff + i]], x0, y0, x1, y1);
    diff_add(my, stride, x0, y0, x1, y1);
  }
  __syncthreads();
  for (int ww = 0; ww < nw; ++ww) {
    int* d = wd + ww * maxcells;
    for (int y = w; y <= gy; y += 4) wave_prefix(d + y * stride, 1, gx + 1);
    __syncthreads();
    for (int x = w; x <= gx; x += 4) wave_prefix(d + x, stride, gy + 1);
    __syncthreads();
  }
  // chunk counts per tile -> local offsets (exclusive scan over tiles)
  const uint32_t* cmv = cm + pt.cm_off[v];
  const int PER = (T + GS_BLOCK - 1) / GS_BLOCK;
  uint32_t local = 0;
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x * PER + k;
    if (t < T) {
      const int ty = t / gx, tx = t - ty * gx, cell = ty * stride + tx;
      for (int ww = 0; ww < nw; ++ww) local += (uint32_t)wd[ww * maxcells + cell];
    }
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(local, s_wave, tot);
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x * PER + k;
    if (t < T) {
      const int ty = t / gx, tx = t - ty * gx, cell = ty * stride + tx;
      lo[t] = (int)run;
      gst[t] = cmv[(int64_t)t * nchunk + c];
      uint32_t p = run;
      for (int ww = 0; ww < nw; ++ww) {
        const int cn = wd[ww * maxcells + cell];
        wd[ww * maxcells + cell] = (int)p;
        p += (uint32_t)cn;
      }
      run = p;
    }
  }
  __syncthreads();
  // wave-serial placement in record order
  for (uint32_t i0 = wlo; i0 < whi; i0 += 64) {
    const uint32_t i = i0 + lane;
    uint32_t id = 0;
    int2 rc = make_int2(1 | (1 << 16), 0);
    if (i < whi) {
      id = sorted[roff + i];
      rc = rect[roff + id];
    }
    const int cnt = (int)min(64u, whi - i0);
    for (int j = 0; j < cnt; ++j) {
      const uint32_t gid = __builtin_amdgcn_readlane(id, j);
      int x0, y0, x1, y1;
      rect_of(make_int2(__builtin_amdgcn_readlane(rc.x, j), __builtin_amdgcn_readlane(rc.y, j)), x0, y0, x1, y1);
      if (x0 > x1) continue;
      const int wdt = x1 - x0 + 1;
      const int n = wdt * (y1 - y0 + 1);
      const float inv = 1.0f / (float)wdt;
      for (int e = lane; e < n; e += 64) {
        const int dy = (int)(((float)e + 0.5f) * inv);
        const int dx = e - dy * wdt;
        const int tx = x0 + dx, ty = y0 + dy;
        const int cell = ty * stride + tx;
        const int p = my[cell];
        my[cell] = p + 1;
        ent[p] = gid;
        etile[p] = (uint16_t)(ty * gx + tx);
      }
    }
  }
  __syncthreads();
  // contiguous copy-out
  for (uint32_t i = threadIdx.x; i < tot; i += GS_BLOCK) {
    const int t = etile[i];
    out_ids[gst[t] + (i - (uint32_t)lo[t])] = ent[i];
  }
  (void)n_inst;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ------------------------------------------------------------------ host side
struct PrefWs {
  size_t theta, nsel, cnt, ka, ia, kb, ib, cb, nchunk, cm, part, bytes;
  int nb_max, maxchunk;
  int64_t cm_n, part_n;
};

// LDS plan of the scatter: `nw` placement waves (each with its own tile
// counter table), the tile tables and up to cap_entries staged entries, within
// the workgroup LDS limit. Returns the chunk budget (instances before the
// record that closes a chunk) or 0 when no plan fits.
static int pref_budget(const ViewTab& tab, size_t lds_limit, int& maxT, int& maxcells, int& cap_entries, size_t& lds,
                       int& nw) {
  maxT = 0;
  maxcells = 0;
  for (int v = 0; v < tab.nv; ++v) {
    maxT = max(maxT, tab.gx[v] * tab.gy[v]);
    maxcells = max(maxcells, (tab.gx[v] + 1) * (tab.gy[v] + 1));
  }
  const size_t limit = lds_limit - 512;  // static shared memory of the kernel
  for (nw = 4; nw >= 1; nw >>= 1) {
    const size_t fixed = (size_t)nw * maxcells * 4 + (size_t)maxT * 8;
    if (fixed >= limit) continue;
    cap_entries = (int)min((size_t)16384, (limit - fixed) / 6);
    cap_entries &= ~63;
    if (cap_entries >= 2 * maxT + 256) {
      lds = fixed + (size_t)cap_entries * 6;
      return cap_entries - maxT;  // a chunk closes before the record that crosses this
    }
  }
  nw = 0;
  cap_entries = 0;
  lds = 0;
  return 0;
}

static PrefWs pref_layout(const ViewTab& tab, size_t lds_limit, int64_t capacity, PrefTab* pt) {
  PrefWs L;
  int maxT, maxcells, cap, nw;
  size_t lds;
  int budget = pref_budget(tab, lds_limit, maxT, maxcells, cap, lds, nw);
  if (budget <= 0) budget = 1;
  int64_t nbm = 0;
  for (int v = 0; v < tab.nv; ++v) nbm = max(nbm, (tab.npad[v] + SEL_TILE - 1) / SEL_TILE);
  L.nb_max = (int)max((int64_t)1, nbm);
  L.maxchunk = (int)min((int64_t)1 << 30, capacity / budget + 2);
  int64_t cm = 0, parts = 0;
  if (pt) {
    pt->maxchunk = L.maxchunk;
    pt->budget = budget;
  }
  for (int v = 0; v < tab.nv; ++v) {
    const int64_t len = (int64_t)tab.gx[v] * tab.gy[v] * L.maxchunk;
    const int nbs = (int)((len + SCAN_TILE2 - 1) / SCAN_TILE2);
    if (pt) {
      pt->cm_off[v] = cm;
      pt->part_off[v] = parts;
      pt->nbs[v] = nbs;
    }
    cm += len;
    parts += nbs;
  }
  L.cm_n = cm;
  L.part_n = parts;
  const size_t M = (size_t)tab.nrec;
  size_t o = 0;
  L.theta = o; o += al256(4 * GS_MAX_VIEWS);
  L.nsel = o; o += al256(4 * GS_MAX_VIEWS);
  L.cnt = o; o += al256((size_t)tab.nv * L.nb_max * 4);
  L.ka = o; o += al256(M * 4);
  L.ia = o; o += al256(M * 4);
  L.kb = o; o += al256(M * 4);
  L.ib = o; o += al256(M * 4);
  L.cb = o; o += al256((size_t)tab.nv * (L.maxchunk + 1) * 4);
  L.nchunk = o; o += al256(4 * GS_MAX_VIEWS);
  L.cm = o; o += al256((size_t)cm * 4);
  L.part = o; o += al256((size_t)parts * 4 + 4);
  L.bytes = o;
  return L;
}

// Workgroup LDS limit for the scatter: the device's per-block maximum when the
// kernel's dynamic limit can be raised to it, else 64 KB. Decided once per
// context (also by the workspace query, so both use the same plan).
static size_t lds_limit_of(gs_ctx* ctx) {
  if (ctx->lds_limit == 0) {
    int v = 0;
    size_t lim = 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) == hipSuccess &&
        v > 65536) {
      if (hipFuncSetAttribute((const void*)pscatter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, v - 512) ==
          hipSuccess)
        lim = (size_t)v;
      else
        (void)hipGetLastError();
    } else {
      (void)hipGetLastError();
    }
    ctx->lds_limit = lim;
  }
  return ctx->lds_limit;
}

size_t bin_prefix_ws_bytes(gs_ctx* ctx, const ViewTab& tab, int64_t capacity) {
  return pref_layout(tab, lds_limit_of(ctx), capacity, nullptr).bytes;
}

gs_status launch_bin_prefix(gs_ctx* ctx, const ViewTab& tab, const gs_camera* cams, const gs_gaussians* g,
                            const gs_proj* proj, gs_bins* bins, char* ws, hipStream_t s) {
  PrefTab pt;
  GaussSrc gsrc;
  gsrc.mean = g->mean;
  gsrc.log_scale = g->log_scale;
  gsrc.quat = g->quat;
  gsrc.opl = g->opacity_logit;
  gsrc.color = g->color;
  gsrc.mp = g->mp;
  gsrc.n = g->n;
  const size_t lim = lds_limit_of(ctx);
  const PrefWs L = pref_layout(tab, lim, bins->capacity, &pt);
  int maxT, maxcells, cap, nw;
  size_t lds;
  if (pref_budget(tab, lim, maxT, maxcells, cap, lds, nw) <= 0)
    return gs_fail(ctx, GS_E_UNSUPPORTED, "image too large for the prefix binning LDS plan (%zu B limit)", lim);
  uint32_t* theta = (uint32_t*)(ws + L.theta);
  uint32_t* nsel = (uint32_t*)(ws + L.nsel);
  uint32_t* cnt = (uint32_t*)(ws + L.cnt);
  uint32_t* ka = (uint32_t*)(ws + L.ka);
  uint32_t* ia = (uint32_t*)(ws + L.ia);
  uint32_t* kb = (uint32_t*)(ws + L.kb);
  uint32_t* ib = (uint32_t*)(ws + L.ib);
  uint32_t* cb = (uint32_t*)(ws + L.cb);
  uint32_t* nchunk = (uint32_t*)(ws + L.nchunk);
  uint32_t* cm = (uint32_t*)(ws + L.cm);
  uint32_t* part = (uint32_t*)(ws + L.part);
  const int2* rect = (const int2*)proj->rect;
  const dim3 gsel(L.nb_max, tab.nv);
  GS_LAUNCH(ctx, sel_count_kernel, gsel, dim3(GS_BLOCK), 0, s, tab, proj->depth_key, proj->key_hist,
            bins->max_rank, L.nb_max, theta, cnt, bins->overflow);
  GS_LAUNCH(ctx, compact_kernel, gsel, dim3(GS_BLOCK), 0, s, tab, proj->depth_key, theta, cnt, L.nb_max,
            proj->key_hist, ka, ia, nsel);
  GS_LAUNCH(ctx, sel_sort_kernel, dim3(tab.nv), dim3(SORT_THREADS), 0, s, tab, ka, ia, kb, ib, nsel, rect,
            bins->sorted_ids, pt.budget, L.maxchunk, cb, nchunk, bins->capacity, bins->overflow);
  const int gch = ((L.maxchunk + 7) >> 3) << 3;
  GS_LAUNCH(ctx, pcount_kernel, dim3(gch, tab.nv), dim3(GS_BLOCK), (size_t)maxcells * 4, s, tab, pt, cb, nchunk,
            bins->sorted_ids, rect, cm, cams, gsrc, (float4*)proj->rec);
  int nbs_max = 1;
  for (int v = 0; v < tab.nv; ++v) nbs_max = max(nbs_max, pt.nbs[v]);
  GS_LAUNCH(ctx, pscan_reduce_kernel, dim3(nbs_max, tab.nv), dim3(GS_BLOCK), 0, s, tab, pt, nchunk, cm, part);
  GS_LAUNCH(ctx, pscan_apply_kernel, dim3(nbs_max, tab.nv), dim3(GS_BLOCK), 0, s, tab, pt, nchunk, cm, part,
            L.part_n, bins->capacity, bins->tile_start, bins->n_instances, bins->overflow, bins->incomplete);
  GS_LAUNCH(ctx, pscatter_kernel, dim3(gch, tab.nv), dim3(GS_BLOCK), lds, s, tab, pt, cb, nchunk, bins->sorted_ids,
            rect, cm, bins->n_instances, bins->overflow, bins->gauss_id, maxT, maxcells, cap, nw);
  return gs_check_launch(ctx, "bin_sort (prefix)");
}
