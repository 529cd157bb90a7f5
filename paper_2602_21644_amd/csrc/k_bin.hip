// gs_bin_sort: per-view LSD radix sort of the records' depth keys, then tile
// binning in that order by count -> exclusive scan -> scatter over chunks.
//
// Result: for every tile the ids of the records whose tile rect contains it,
// in ascending (depth bits, id) order. This is exactly the stable sort of the
// (tile << 32 | depth bits) keys: the depth sort is stable and starts from id
// order, and the tile pass places each chunk's instances after those of all
// earlier chunks and, inside a chunk, in record order (each wave walks its
// records one at a time).
#include "bin_common.h"

namespace {

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = GS_BLOCK * SORT_ITEMS;  // keys per radix block
constexpr int SCAN_TILE = 4096;                   // elements per scan block

__global__ __launch_bounds__(GS_BLOCK) void scan_reduce_kernel(const uint32_t* __restrict__ a, int64_t n,
                                                               uint32_t* __restrict__ part) {
  __shared__ uint32_t s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  uint32_t sum = 0;
  for (int i = threadIdx.x; i < SCAN_TILE; i += GS_BLOCK) {
    const int64_t j = base + i;
    if (j < n) sum += a[j];
  }
  uint32_t tot;
  block_excl_scan(sum, s_wave, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block partials; writes the grand total.
__global__ __launch_bounds__(GS_BLOCK) void scan_partials_kernel(uint32_t* __restrict__ part, int64_t nb,
                                                                 int64_t* __restrict__ total_out) {
  __shared__ uint32_t s_wave[4];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += GS_BLOCK) {
    const int64_t j = b0 + threadIdx.x;
    const uint32_t x = j < nb ? part[j] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(x, s_wave, tot);
    if (j < nb) part[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = (int64_t)carry;
}

__global__ __launch_bounds__(GS_BLOCK) void scan_apply_kernel(uint32_t* __restrict__ a, int64_t n,
                                                              const uint32_t* __restrict__ part) {
  __shared__ uint32_t s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  // each thread owns 16 consecutive elements
  constexpr int PER = SCAN_TILE / GS_BLOCK;
  uint32_t vals[PER];
  uint32_t sum = 0;
  const int64_t my = base + (int64_t)threadIdx.x * PER;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    vals[i] = (my + i < n) ? a[my + i] : 0u;
    sum += vals[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(sum, s_wave, tot) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (my + i < n) a[my + i] = run;
    run += vals[i];
  }
}

gs_status exclusive_scan(gs_ctx* ctx, uint32_t* a, int64_t n, uint32_t* part, int64_t* total, hipStream_t s) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 0) return GS_OK;
  GS_LAUNCH(ctx, scan_reduce_kernel, dim3((unsigned)nb), dim3(GS_BLOCK), 0, s, a, n, part);
  GS_LAUNCH(ctx, scan_partials_kernel, dim3(1), dim3(GS_BLOCK), 0, s, part, nb, total);
  GS_LAUNCH(ctx, scan_apply_kernel, dim3((unsigned)nb), dim3(GS_BLOCK), 0, s, a, n, part);
  return gs_check_launch(ctx, "scan");
}

// ------------------------------------------------------------------ radix sort of depth keys
// Histogram of one 8-bit digit per block; stored digit-major per view so that
// one exclusive scan over all views yields every block's output base.
__global__ __launch_bounds__(GS_BLOCK) void radix_hist_kernel(ViewTab tab, BinTab bt,
                                                              const uint32_t* __restrict__ keys, int shift,
                                                              uint32_t* __restrict__ hist) {
  const int v = blockIdx.y, b = blockIdx.x;
  if (b >= bt.sblk[v]) return;
  __shared__ uint32_t h[RADIX];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)b * SORT_TILE;
  const int64_t npad = tab.npad[v];
  const uint32_t* kv = keys + tab.r_off[v];
#pragma unroll
  for (int i = 0; i < SORT_ITEMS; ++i) {
    const int64_t j = base + i * GS_BLOCK + threadIdx.x;
    if (j < npad) atomicAdd(&h[(kv[j] >> shift) & (RADIX - 1)], 1u);
  }
  __syncthreads();
  hist[bt.h_off[v] + (int64_t)threadIdx.x * bt.sblk[v] + b] = h[threadIdx.x];
}

// Stable scatter: items are visited in rounds of 256 consecutive keys; inside
// a round a key's rank is (keys of its digit in earlier rounds) + (in earlier
// waves of this round) + (in lower lanes of its wave).
__global__ __launch_bounds__(GS_BLOCK) void radix_scatter_kernel(ViewTab tab, BinTab bt,
                                                                 const uint32_t* __restrict__ kin,
                                                                 const uint32_t* __restrict__ vin,
                                                                 uint32_t* __restrict__ kout,
                                                                 uint32_t* __restrict__ vout, int shift,
                                                                 const uint32_t* __restrict__ hist) {
  const int v = blockIdx.y, b = blockIdx.x;
  if (b >= bt.sblk[v]) return;
  __shared__ uint32_t s_base[RADIX];
  __shared__ uint32_t s_wcnt[4][RADIX];
  __shared__ uint32_t s_woff[4][RADIX];
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  s_base[threadIdx.x] = hist[bt.h_off[v] + (int64_t)threadIdx.x * bt.sblk[v] + b];
  for (int i = 0; i < 4; ++i) s_wcnt[i][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)b * SORT_TILE;
  const int64_t npad = tab.npad[v];
  const int64_t roff = tab.r_off[v];
  const uint64_t lt = lanemask_lt();
  for (int round = 0; round < SORT_ITEMS; ++round) {
    const int64_t j = base + round * GS_BLOCK + threadIdx.x;
    const bool valid = j < npad;
    const uint32_t key = valid ? kin[roff + j] : 0u;
    const uint32_t val = valid ? (vin ? vin[roff + j] : (uint32_t)j) : 0u;
    const uint32_t d = (key >> shift) & (RADIX - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < RADIX_BITS; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt);
    if (valid && rank == 0) s_wcnt[w][d] = __popcll(peers);
    __syncthreads();
    {
      const int dd = threadIdx.x;
      uint32_t o = s_base[dd];
      for (int i = 0; i < 4; ++i) {
        const uint32_t c = s_wcnt[i][dd];
        s_woff[i][dd] = o;
        o += c;
        s_wcnt[i][dd] = 0;
      }
      s_base[dd] = o;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = s_woff[w][d] + rank;  // global record index
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
  (void)lane;
}

__global__ __launch_bounds__(GS_BLOCK) void bin_count_kernel(ViewTab tab, BinTab bt,
                                                             const uint32_t* __restrict__ sorted,
                                                             const int2* __restrict__ rect,
                                                             const uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ cm) {
  extern __shared__ int s_diff[];
  const int v = blockIdx.y;
  const int nchunk = bt.nchunk[v];
  const int gridx = ((nchunk + 7) >> 3) << 3;
  if ((int)blockIdx.x >= gridx) return;
  const int c = chunk_of_block(blockIdx.x, nchunk);
  if (c >= nchunk) return;
  const int gx = tab.gx[v], gy = tab.gy[v];
  const int cells = (gx + 1) * (gy + 1);
  for (int i = threadIdx.x; i < cells; i += GS_BLOCK) s_diff[i] = 0;
  __syncthreads();
  const int64_t roff = tab.r_off[v];
  const int64_t lo = (int64_t)c * bt.chunk;
  const int64_t hi = min(lo + bt.chunk, bt.nlim[v]);
  for (int64_t i = lo + threadIdx.x; i < hi; i += GS_BLOCK) {
    const uint32_t id = sorted[roff + i];
    const int64_t r = roff + id;
    if (key[r] == 0xFFFFFFFFu) continue;
    int x0, y0, x1, y1;
    if (!rect_clip(rect[r], gx, gy, x0, y0, x1, y1)) continue;
    diff_add(s_diff, gx + 1, x0, y0, x1, y1);
  }
  __syncthreads();
  diff_integrate(s_diff, gx, gy, threadIdx.x >> 6, GS_BLOCK / 64);
  const int T = gx * gy;
  uint32_t* out = cm + bt.cm_off[v] + c;
  for (int t = threadIdx.x; t < T; t += GS_BLOCK) {
    const int ty = t / gx, tx = t - ty * gx;
    out[(int64_t)t * nchunk] = (uint32_t)s_diff[ty * (gx + 1) + tx];
  }
}

__global__ __launch_bounds__(GS_BLOCK) void bin_ranges_kernel(ViewTab tab, BinTab bt, const uint32_t* __restrict__ cm,
                                                              const int64_t* __restrict__ total,
                                                              int64_t capacity, uint32_t* __restrict__ tile_start,
                                                              int64_t* __restrict__ n_inst,
                                                              int32_t* __restrict__ overflow,
                                                              int32_t* __restrict__ incomplete,
                                                              const uint32_t* __restrict__ sorted,
                                                              const uint32_t* __restrict__ key,
                                                              int32_t* __restrict__ trunc,
                                                              int32_t* __restrict__ sticky) {
  const int t = blockIdx.x * GS_BLOCK + threadIdx.x;
  if (t < tab.ntiles) {
    const int v = view_of_tile(tab, t);
    const int lt = t - tab.tile_base[v];
    tile_start[t] = cm[bt.cm_off[v] + (int64_t)lt * bt.nchunk[v]];
  }
  if (t == 0) {
    const int64_t tot = *total;
    tile_start[tab.ntiles] = (uint32_t)tot;
    *n_inst = tot;
    *overflow = tot > capacity ? 1 : 0;
    if (sticky && tot > capacity) atomicOr(&sticky[0], 1);
    if (incomplete) *incomplete = 0;
    if (trunc) {
      // a view binned only its first nlim sorted records leaves out a visible
      // one when the first record past the limit is visible (culled records
      // sort last)
      int32_t bits = 0;
      for (int v = 0; v < tab.nv; ++v) {
        if (!bt.truncated[v]) continue;
        const int64_t roff = tab.r_off[v];
        if (key[roff + sorted[roff + bt.nlim[v]]] != 0xFFFFFFFFu) bits |= 1 << v;
      }
      *trunc = bits;
    }
  }
}

// Scatter. Wave w of block (view v, chunk c) owns records [c*chunk + w*chunk/4,
// + chunk/4) in sorted order. Its running write position per tile starts at
// the scanned count of (tile, chunk) plus the counts of lower waves, and it
// walks its records one at a time, lanes covering the record's tiles.
__global__ __launch_bounds__(GS_BLOCK) void bin_scatter_kernel(ViewTab tab, BinTab bt,
                                                               const uint32_t* __restrict__ sorted,
                                                               const int2* __restrict__ rect,
                                                               const uint32_t* __restrict__ key,
                                                               const uint32_t* __restrict__ cm,
                                                               const int32_t* __restrict__ overflow,
                                                               uint32_t* __restrict__ out_ids) {
  extern __shared__ int s_mem[];
  if (*overflow) return;
  const int v = blockIdx.y;
  const int nchunk = bt.nchunk[v];
  const int gridx = ((nchunk + 7) >> 3) << 3;
  if ((int)blockIdx.x >= gridx) return;
  const int c = chunk_of_block(blockIdx.x, nchunk);
  if (c >= nchunk) return;
  const int gx = tab.gx[v], gy = tab.gy[v];
  const int stride = gx + 1;
  const int cells = stride * (gy + 1);
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  int* my = s_mem + w * cells;
  for (int i = threadIdx.x; i < 4 * cells; i += GS_BLOCK) s_mem[i] = 0;
  __syncthreads();
  const int64_t roff = tab.r_off[v];
  const int per_wave = bt.chunk >> 2;
  const int64_t lo = (int64_t)c * bt.chunk + (int64_t)w * per_wave;
  const int64_t hi = min(lo + per_wave, bt.nlim[v]);
  for (int64_t i = lo + lane; i < hi; i += 64) {
    const uint32_t id = sorted[roff + i];
    const int64_t r = roff + id;
    if (key[r] == 0xFFFFFFFFu) continue;
    int x0, y0, x1, y1;
    if (!rect_clip(rect[r], gx, gy, x0, y0, x1, y1)) continue;
    diff_add(my, stride, x0, y0, x1, y1);
  }
  __syncthreads();
  for (int ww = 0; ww < 4; ++ww) {
    // integrate wave ww's array with all 4 waves (rows then columns)
    int* d = s_mem + ww * cells;
    for (int y = w; y <= gy; y += 4) wave_prefix(d + y * stride, 1, gx + 1);
    __syncthreads();
    for (int x = w; x <= gx; x += 4) wave_prefix(d + x, stride, gy + 1);
    __syncthreads();
  }
  // per-tile start positions of each wave
  const int T = gx * gy;
  const uint32_t* cmv = cm + bt.cm_off[v] + c;
  for (int t = threadIdx.x; t < T; t += GS_BLOCK) {
    const int ty = t / gx, tx = t - ty * gx;
    const int cell = ty * stride + tx;
    uint32_t pos = cmv[(int64_t)t * nchunk];
    for (int ww = 0; ww < 4; ++ww) {
      const uint32_t cnt = (uint32_t)s_mem[ww * cells + cell];
      s_mem[ww * cells + cell] = (int)pos;
      pos += cnt;
    }
  }
  __syncthreads();
  // wave-serial emission in sorted order
  for (int64_t i0 = lo; i0 < hi; i0 += 64) {
    const int64_t i = i0 + lane;
    uint32_t id = 0;
    int2 rc = make_int2(1 | (1 << 16), 0);
    if (i < hi) {
      id = sorted[roff + i];
      const int64_t r = roff + id;
      if (key[r] != 0xFFFFFFFFu) rc = rect[r];
    }
    const int cnt = (int)min((int64_t)64, hi - i0);
    for (int j = 0; j < cnt; ++j) {
      const uint32_t gid = __builtin_amdgcn_readlane(id, j);
      const int rx = __builtin_amdgcn_readlane(rc.x, j);
      const int ry = __builtin_amdgcn_readlane(rc.y, j);
      int x0, y0, x1, y1;
      if (!rect_clip(make_int2(rx, ry), gx, gy, x0, y0, x1, y1)) continue;
      const int wdt = x1 - x0 + 1;
      const int n = wdt * (y1 - y0 + 1);
      for (int e = lane; e < n; e += 64) {
        const int dy = e / wdt;
        const int dx = e - dy * wdt;
        const int cell = (y0 + dy) * stride + (x0 + dx);
        const int p = my[cell];
        my[cell] = p + 1;
        out_ids[(uint32_t)p] = gid;
      }
    }
  }
}

}  // namespace

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

BinWs bin_ws_layout(const ViewTab& tab, const BinTab& bt) {
  BinWs L;
  size_t o = 0;
  const size_t M = (size_t)tab.nrec;
  L.keys_a = o; o += al256(M * 4);
  L.keys_b = o; o += al256(M * 4);
  L.vals_a = o; o += al256(M * 4);
  L.vals_b = o; o += al256(M * 4);
  int64_t hn = 0, cn = 0;
  for (int v = 0; v < tab.nv; ++v) {
    hn += (int64_t)RADIX * bt.sblk[v];
    cn += (int64_t)tab.gx[v] * tab.gy[v] * bt.nchunk[v];
  }
  L.hist_n = hn;
  L.cm_n = cn;
  L.hist = o; o += al256((size_t)hn * 4);
  const int64_t maxn = hn > cn ? hn : cn;
  L.part = o; o += al256((size_t)((maxn + SCAN_TILE - 1) / SCAN_TILE + 1) * 4);
  L.total = o; o += al256(16);
  L.cm = o; o += al256((size_t)cn * 4);
  L.bytes = o;
  return L;
}

void bin_tab_fill(const ViewTab& tab, int chunk, int64_t max_rank, BinTab& bt) {
  bt.chunk = chunk;
  int64_t cm = 0, h = 0;
  for (int v = 0; v < tab.nv; ++v) {
    const int64_t np = tab.npad[v];
    const int64_t lim = (max_rank > 0 && max_rank < np) ? max_rank : np;
    bt.nlim[v] = lim;
    bt.truncated[v] = lim < np ? 1 : 0;
    int64_t nc = (lim + chunk - 1) / chunk;
    if (nc < 1) nc = 1;
    bt.nchunk[v] = (int32_t)nc;
    bt.cm_off[v] = cm;
    cm += (int64_t)tab.gx[v] * tab.gy[v] * nc;
    bt.sblk[v] = (int32_t)((np + SORT_TILE - 1) / SORT_TILE);
    bt.h_off[v] = h;
    h += (int64_t)RADIX * bt.sblk[v];
  }
}

size_t bin_lds_bytes(const ViewTab& tab) {
  int maxc = 0;
  for (int v = 0; v < tab.nv; ++v) {
    const int c = (tab.gx[v] + 1) * (tab.gy[v] + 1);
    maxc = c > maxc ? c : maxc;
  }
  return (size_t)maxc * 4 * 4;
}

gs_status launch_bin_sort(gs_ctx* ctx, const ViewTab& tab, const BinTab& bt, const gs_proj* proj, gs_bins* bins,
                          char* ws, hipStream_t s) {
  const BinWs L = bin_ws_layout(tab, bt);
  uint32_t* ka = (uint32_t*)(ws + L.keys_a);
  uint32_t* kb = (uint32_t*)(ws + L.keys_b);
  uint32_t* va = (uint32_t*)(ws + L.vals_a);
  uint32_t* vb = (uint32_t*)(ws + L.vals_b);
  uint32_t* hist = (uint32_t*)(ws + L.hist);
  uint32_t* part = (uint32_t*)(ws + L.part);
  int64_t* total = (int64_t*)(ws + L.total);
  uint32_t* cm = (uint32_t*)(ws + L.cm);
  int maxblk = 0, maxchunk = 0;
  for (int v = 0; v < tab.nv; ++v) {
    maxblk = bt.sblk[v] > maxblk ? bt.sblk[v] : maxblk;
    const int g8 = ((bt.nchunk[v] + 7) >> 3) << 3;
    maxchunk = g8 > maxchunk ? g8 : maxchunk;
  }
  // 4 stable 8-bit passes: keys ping-pong depth_key -> a -> b -> a -> b;
  // the last pass writes the ids straight into bins->sorted_ids.
  const uint32_t* kin = proj->depth_key;
  const uint32_t* vin = nullptr;
  uint32_t* kouts[4] = {ka, kb, ka, kb};
  uint32_t* vouts[4] = {va, vb, va, bins->sorted_ids};
  if (maxblk > 0) {
    for (int pass = 0; pass < 4; ++pass) {
      const int shift = pass * RADIX_BITS;
      GS_LAUNCH(ctx, radix_hist_kernel, dim3(maxblk, tab.nv), dim3(GS_BLOCK), 0, s, tab, bt, kin, shift, hist);
      gs_status st = exclusive_scan(ctx, hist, L.hist_n, part, nullptr, s);
      if (st != GS_OK) return st;
      GS_LAUNCH(ctx, radix_scatter_kernel, dim3(maxblk, tab.nv), dim3(GS_BLOCK), 0, s, tab, bt, kin, vin,
                         kouts[pass], vouts[pass], shift, hist);
      kin = kouts[pass];
      vin = vouts[pass];
    }
  }
  const size_t lds = bin_lds_bytes(tab);
  GS_LAUNCH(ctx, bin_count_kernel, dim3(maxchunk, tab.nv), dim3(GS_BLOCK), lds / 4, s, tab, bt,
                     bins->sorted_ids, (const int2*)proj->rect, proj->depth_key, cm);
  gs_status st = exclusive_scan(ctx, cm, L.cm_n, part, total, s);
  if (st != GS_OK) return st;
  GS_LAUNCH(ctx, bin_ranges_kernel, dim3((tab.ntiles + GS_BLOCK) / GS_BLOCK), dim3(GS_BLOCK), 0, s, tab, bt, cm,
                     total, bins->capacity, bins->tile_start, bins->n_instances, bins->overflow, bins->incomplete,
                     bins->sorted_ids, proj->depth_key, bins->max_rank > 0 ? bins->truncated : nullptr,
                     bins->sticky);
  GS_LAUNCH(ctx, bin_scatter_kernel, dim3(maxchunk, tab.nv), dim3(GS_BLOCK), lds, s, tab, bt,
                     bins->sorted_ids, (const int2*)proj->rect, proj->depth_key, cm, bins->overflow,
                     bins->gauss_id);
  return gs_check_launch(ctx, "bin_sort");
}
