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
// and the caller re-bins with a larger rank or the full path.
//
// The selection is small (thousands of records), so the path is built for
// that size:
//   psel:   one pass over the keys; the selected records of each 2048-record
//           block go to the block's own segment (no global scan) and get their
//           48-byte compositing record;
//   psort:  one 1024-thread workgroup per view gathers the segments into
//           registers, sorts them on (key, id) in LDS (counting pass on the top
//           12 bits of the key range, then each record's rank inside its
//           bucket, or a bitonic network for a bucket of thousands of
//           records), writes the sorted ids and rects and the view's instance
//           total (the sum of the rect areas);
//   ptiles: a workgroup per 2x2 block of tiles keeps, in order, the sorted
//           records that meet the block (in LDS) and finds where each of its
//           tile lists starts: the instances in front of tile t in row-major
//           order, summed over the records in closed form (rows of the rect
//           above t times its width, plus its columns left of t in t's row).
//           Then one wave per tile appends the ids that cover its tile.
// A view whose selection exceeds PS_CAP records gets empty lists and raises
// `incomplete`.
#include "bin_common.h"
#include "gs_project_dev.h"

namespace {

constexpr int HB = 4096;                        // coarse histogram bins
constexpr int SEL_ITEMS = 8;
constexpr int SEL_TILE = GS_BLOCK * SEL_ITEMS;  // records per selection block
constexpr int PS_THREADS = 1024;
constexpr int PS_CAP = 12288;                   // selected records per view
constexpr int PS_PER = PS_CAP / PS_THREADS;
constexpr int PS_BUCKETS = 4096;
// buckets larger than this are sorted by a network instead of being ranked
// record by record (at most PS_CAP / (PS_BIG + 1) of them). A network stage
// with its workgroup barrier costs ~1000 cycles, so the network only pays
// for buckets of several thousand records: one of 561 took 58k cycles
// sorted, 63k ranked.
constexpr int PS_BIG = 4096;
constexpr int PS_MAXBIG = PS_CAP / (PS_BIG + 1) + 1;
static_assert(PS_CAP < 0xFFFF, "0xFFFF marks a slot outside the sorted buckets");
constexpr int PS_MAXBLK = 4096;                 // selection blocks per view (8.4M records)
// dynamic LDS of psort: keys and ids grouped by bucket, bucket cursors, the
// block offsets (later the bucket starts), and the final position of each
// bucket slot (16 bits)
constexpr size_t PS_LDS =
    (size_t)PS_CAP * 8 + (size_t)PS_BUCKETS * 4 + (size_t)(PS_MAXBLK + 1) * 4 + (size_t)PS_CAP * 2;
static_assert(PS_CAP <= 65536, "final positions are 16-bit");
static_assert(PS_BUCKETS == 4 * PS_THREADS && PS_MAXBLK == 4 * PS_THREADS, "4 entries per thread");

__device__ __forceinline__ int sel_blocks(int64_t npad) { return (int)((npad + SEL_TILE - 1) / SEL_TILE); }

// Threshold from the coarse histogram of one view: keys < theta are selected.
__device__ uint32_t theta_of(const uint32_t* __restrict__ hist, int64_t R, uint32_t* s_wave, uint32_t& total) {
  __shared__ uint32_t s_theta;
  constexpr int PER = HB / GS_BLOCK;
  uint32_t loc[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    loc[i] = hist[threadIdx.x * PER + i];
    sum += loc[i];
  }
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

__global__ __launch_bounds__(GS_BLOCK) void psel_kernel(ViewTab tab, const uint32_t* __restrict__ key,
                                                        const uint32_t* __restrict__ hist,
                                                        const int2* __restrict__ rect, int64_t R, int nb_max,
                                                        const gs_camera* __restrict__ cams, GaussSrc gsrc,
                                                        float4* __restrict__ rec, uint32_t* __restrict__ seg_key,
                                                        uint32_t* __restrict__ seg_id, int2* __restrict__ seg_rect,
                                                        uint32_t* __restrict__ cnt, int32_t* __restrict__ overflow,
                                                        int32_t* __restrict__ incomplete, int32_t* __restrict__ trunc,
                                                        uint32_t* __restrict__ nvis, int keys_only) {
  __shared__ uint32_t s_wave[4];
  __shared__ uint32_t s_n;
  __shared__ uint32_t s_sel[SEL_TILE];
  const int v = blockIdx.y, b = blockIdx.x;
  if (v == 0 && b == 0 && threadIdx.x == 0) {
    *overflow = 0;
    *incomplete = 0;
    *trunc = 0;
  }
  const int64_t npad = tab.npad[v];
  if (b >= sel_blocks(npad)) return;  // uniform per workgroup
  const int64_t roff = tab.r_off[v];
  // the block's keys are in flight while the threshold is found
  uint32_t kk[SEL_ITEMS];
#pragma unroll
  for (int i = 0; i < SEL_ITEMS; ++i) {
    const int64_t j = (int64_t)b * SEL_TILE + i * GS_BLOCK + threadIdx.x;
    kk[i] = j < npad ? key[roff + j] : 0xFFFFFFFFu;
  }
  uint32_t visible;
  const uint32_t theta = theta_of(hist + (int64_t)v * HB, R, s_wave, visible);
  if (threadIdx.x == 0) {
    s_n = 0;
    if (b == 0) nvis[v] = visible;  // the view's visible records
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  const int64_t sbase = roff + (int64_t)b * SEL_TILE;
#pragma unroll
  for (int i = 0; i < SEL_ITEMS; ++i) {
    const uint32_t j = (uint32_t)(b * SEL_TILE + i * GS_BLOCK + threadIdx.x);
    const bool s = kk[i] != 0xFFFFFFFFu && kk[i] < theta;
    // wave-aggregated slot in the block's segment (order is irrelevant: psort sorts)
    const uint64_t m = __ballot(s);
    if (m) {
      uint32_t base = 0;
      if (__lane_id() == 0) base = atomicAdd(&s_n, (uint32_t)__popcll(m));
      base = __shfl(base, 0, 64);
      if (s) {
        const uint32_t p = base + __popcll(m & lt);
        seg_key[sbase + p] = kk[i];
        seg_id[sbase + p] = j;
        s_sel[p] = j;
      }
    }
  }
  __syncthreads();
  const uint32_t ns = s_n;
  if (threadIdx.x == 0) cnt[(int64_t)v * nb_max + b] = ns;
  // exact projection of every selected record, one per thread: its
  // compositing record and, when gs_project wrote the depth keys only, its
  // tile rect (empty when the exact test culls a record the screen test kept,
  // so that it lands in no list)
  const gs_camera cam = cams[v];
  const int64_t N = gsrc.n;
  for (uint32_t p = threadIdx.x; p < ns; p += GS_BLOCK) {
    const uint32_t j = s_sel[p];
    const int64_t gk = tab.g_off[v] + j;
    const float m[3] = {gsrc.mean[gk], gsrc.mean[N + gk], gsrc.mean[2 * N + gk]};
    const float ls[3] = {gsrc.log_scale[gk], gsrc.log_scale[N + gk], gsrc.log_scale[2 * N + gk]};
    const float q[4] = {gsrc.quat[gk], gsrc.quat[N + gk], gsrc.quat[2 * N + gk], gsrc.quat[3 * N + gk]};
    const ProjF P = project_f(cam, m, ls, q, gsrc.opl[gk]);
    int2 rc;
    int rr;
    if (keys_only)
      tile_rect_of(P, tab.gx[v], tab.gy[v], rc, rr);
    else
      rc = rect[roff + j];
    seg_rect[sbase + p] = rc;
    rec[3 * (roff + j) + 0] = make_float4(P.ux, P.uy, P.pz, P.o);
    rec[3 * (roff + j) + 1] =
        make_float4(gs_conic_scale_diag(P.k1), gs_conic_scale_off(P.k2), gs_conic_scale_diag(P.k3), gsrc.mp[gk]);
    rec[3 * (roff + j) + 2] = make_float4(gsrc.color[gk], gsrc.color[N + gk], gsrc.color[2 * N + gk], 0.f);
  }
}

// Exclusive scan over the 1024-thread block (16 waves).
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
  for (int i = 0; i < PS_THREADS / 64; ++i) {
    const uint32_t t = s_w[i];
    if (i < w) base += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + inc - x;
}

__global__ __launch_bounds__(PS_THREADS) void psort_kernel(
    ViewTab tab, int nb_max, const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ seg_key,
    const uint32_t* __restrict__ seg_id, const int2* __restrict__ seg_rect, uint32_t* __restrict__ hist,
    uint32_t* __restrict__ sorted_ids, int2* __restrict__ srect, uint32_t* __restrict__ view_total,
    uint32_t* __restrict__ nsel_out, int32_t* __restrict__ incomplete, int32_t* __restrict__ trunc,
    const uint32_t* __restrict__ nvis, int32_t* __restrict__ sticky) {
  extern __shared__ uint32_t s_dyn[];
  uint32_t* gk = s_dyn;              // [PS_CAP] keys grouped by bucket; later the difference array
  uint32_t* gi = gk + PS_CAP;        // [PS_CAP] ids
  uint32_t* cur = gi + PS_CAP;       // [PS_BUCKETS] bucket cursors
  uint32_t* bst = cur + PS_BUCKETS;  // [PS_MAXBLK + 1] block offsets, then bucket starts
  uint16_t* fpos = reinterpret_cast<uint16_t*>(bst + PS_MAXBLK + 1);  // [PS_CAP] final position per slot
  __shared__ uint32_t s_w[PS_THREADS / 64];
  __shared__ uint32_t s_min, s_max, s_area;
  __shared__ uint32_t s_nbig, s_big[PS_MAXBIG];
  __shared__ uint32_t s_bb0[PS_MAXBIG], s_bbn[PS_MAXBIG], s_blp[PS_MAXBIG], s_boff[PS_MAXBIG + 1], s_lmax;
  const int v = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t roff = tab.r_off[v];
  const int nb = sel_blocks(tab.npad[v]);
  // 1. offsets of the block segments
  uint32_t c4[4], s4 = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = tid * 4 + q;
    c4[q] = i < nb ? cnt[(int64_t)v * nb_max + i] : 0u;
    s4 += c4[q];
  }
  uint32_t n;
  uint32_t run = block1024_excl(s4, s_w, n);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    bst[tid * 4 + q] = run;
    run += c4[q];
  }
  if (tid == 0) {
    bst[PS_MAXBLK] = n;
    s_nbig = 0u;
    s_min = 0xFFFFFFFFu;
    s_max = 0u;
    s_area = 0u;
  }
  for (int i = tid; i < HB; i += PS_THREADS) hist[(int64_t)v * HB + i] = 0;  // consumed
  __syncthreads();
  if (n > (uint32_t)PS_CAP) {
    // too many records in front of the threshold for this path: empty lists
    if (tid == 0) {
      view_total[v] = 0;
      nsel_out[v] = 0;
      *incomplete = 1;
      atomicOr(trunc, 1 << v);
      if (sticky) atomicOr(&sticky[1], 1);
    }
    return;
  }
  // the lists leave out a visible record: a tile that runs out of its list
  // with light still passing is not exact (psel counted the visible records
  // of every view with records)
  if (tid == 0 && nb > 0 && n < nvis[v]) atomicOr(trunc, 1 << v);
  // 2. gather into registers: record e lives in the segment of block b with
  //    bst[b] <= e < bst[b + 1]
  uint32_t kr[PS_PER], ir[PS_PER];
  int2 rr[PS_PER];
  int64_t adr[PS_PER];
#pragma unroll
  for (int q = 0; q < PS_PER; ++q) {
    const uint32_t e = (uint32_t)(q * PS_THREADS + tid);
    adr[q] = -1;
    if (e < n) {
      int lo = 0, hi = nb;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bst[mid] <= e) lo = mid;
        else hi = mid;
      }
      adr[q] = roff + (int64_t)lo * SEL_TILE + (e - bst[lo]);
    }
  }
  // every load in flight before any is used
#pragma unroll
  for (int q = 0; q < PS_PER; ++q) {
    kr[q] = adr[q] >= 0 ? seg_key[adr[q]] : 0xFFFFFFFFu;
    ir[q] = adr[q] >= 0 ? seg_id[adr[q]] : 0u;
    rr[q] = adr[q] >= 0 ? seg_rect[adr[q]] : make_int2(1 | (1 << 16), 0);
  }
  uint32_t lmin = 0xFFFFFFFFu, lmax = 0u, larea = 0u;
#pragma unroll
  for (int q = 0; q < PS_PER; ++q) {
    if (adr[q] >= 0) {
      lmin = min(lmin, kr[q]);
      lmax = max(lmax, kr[q]);
      int x0, y0, x1, y1;
      rect_of(rr[q], x0, y0, x1, y1);
      larea += (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lmin = min(lmin, (uint32_t)__shfl_xor((int)lmin, o, 64));
    lmax = max(lmax, (uint32_t)__shfl_xor((int)lmax, o, 64));
    larea += (uint32_t)__shfl_xor((int)larea, o, 64);
  }
  if (__lane_id() == 0) {
    atomicMin(&s_min, lmin);
    atomicMax(&s_max, lmax);
    atomicAdd(&s_area, larea);
  }
  for (int i = tid; i < PS_BUCKETS; i += PS_THREADS) cur[i] = 0;
  __syncthreads();
  const uint32_t kmin = s_min;
  const uint32_t range = n > 0 ? s_max - kmin : 0u;
  const int bits = range ? 32 - __clz(range) : 0;
  const int sh = bits > 12 ? bits - 12 : 0;
  // 3. counting pass over the top 12 bits of (key - kmin)
#pragma unroll
  for (int q = 0; q < PS_PER; ++q)
    if ((uint32_t)(q * PS_THREADS + tid) < n) atomicAdd(&cur[(kr[q] - kmin) >> sh], 1u);
  __syncthreads();
  s4 = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c4[q] = cur[tid * 4 + q];
    s4 += c4[q];
  }
  uint32_t tot;
  run = block1024_excl(s4, s_w, tot);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cur[tid * 4 + q] = run;
    bst[tid * 4 + q] = run;
    run += c4[q];
    if (c4[q] > (uint32_t)PS_BIG) s_big[atomicAdd(&s_nbig, 1u)] = (uint32_t)(tid * 4 + q);
  }
  __syncthreads();
  uint32_t pos[PS_PER];  // each record's slot in bucket order, then its final position
#pragma unroll
  for (int q = 0; q < PS_PER; ++q) {
    pos[q] = 0;
    if ((uint32_t)(q * PS_THREADS + tid) < n) {
      pos[q] = atomicAdd(&cur[(kr[q] - kmin) >> sh], 1u);
      gk[pos[q]] = kr[q];
      gi[pos[q]] = ir[q];
    }
  }
  __syncthreads();
  // 4. Buckets of more than PS_BIG records (many records at nearly one
  //    depth, such as a large surface facing the camera) are sorted in place
  //    on (key, id) by one segmented bitonic network: every bucket's merges
  //    run ascending (the first stage of each compares mirrored positions),
  //    so the positions past a bucket's end act as +inf and their pairs are
  //    skipped, and all such buckets advance through the same stages.
  //    Ranking inside them record by record would take time quadratic in
  //    their size. fpos carries each record's scatter slot through the
  //    network and then maps the slot to its final position.
  const uint32_t nbig = s_nbig;
  if (nbig > 0) {  // uniform
    if (tid == 0) {
      uint32_t off = 0, lmax = 0;
      for (uint32_t bb = 0; bb < nbig; ++bb) {
        const uint32_t d = s_big[bb];
        const uint32_t b0 = bst[d], B = cur[d] - b0;
        uint32_t lp = 0;
        while ((1u << lp) < B) ++lp;
        s_bb0[bb] = b0;
        s_bbn[bb] = B;
        s_blp[bb] = lp;
        s_boff[bb] = off;
        off += 1u << (lp - 1);  // pairs per stage
        lmax = lp > lmax ? lp : lmax;
      }
      s_boff[nbig] = off;
      s_lmax = lmax;
    }
#pragma unroll
    for (int q = 0; q < PS_PER; ++q) {
      const uint32_t i = (uint32_t)(q * PS_THREADS + tid);
      if (i < n) fpos[i] = (uint16_t)i;
    }
    __syncthreads();
    const uint32_t npairs = s_boff[nbig], lmax = s_lmax;
    for (uint32_t lk = 1; lk <= lmax; ++lk) {
      const uint32_t k = 1u << lk;
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
#pragma unroll 1
        for (uint32_t f = tid; f < npairs; f += PS_THREADS) {
          uint32_t bb = 0;
          while (bb + 1 < nbig && s_boff[bb + 1] <= f) ++bb;  // at most PS_MAXBIG steps
          if (lk > s_blp[bb]) continue;                       // this bucket's network is done
          const uint32_t i = f - s_boff[bb], b0 = s_bb0[bb], B = s_bbn[bb];
          uint32_t lo, hi;
          if (j == (k >> 1)) {
            const uint32_t blk = i >> (lk - 1), ps = i & ((k >> 1) - 1u);
            lo = blk * k + ps;
            hi = blk * k + k - 1u - ps;
          } else {
            lo = 2u * i - (i & (j - 1u));
            hi = lo + j;
          }
          if (hi < B) {
            const uint32_t ka = gk[b0 + lo], kb = gk[b0 + hi], ia = gi[b0 + lo], ib = gi[b0 + hi];
            if (ka > kb || (ka == kb && ia > ib)) {
              gk[b0 + lo] = kb;
              gk[b0 + hi] = ka;
              gi[b0 + lo] = ib;
              gi[b0 + hi] = ia;
              const uint16_t t = fpos[b0 + lo];
              fpos[b0 + lo] = fpos[b0 + hi];
              fpos[b0 + hi] = t;
            }
          }
        }
        __syncthreads();
      }
    }
    // in a sorted bucket, slot fpos[x] now sits at x: invert the map there
    uint16_t from[PS_PER];
#pragma unroll
    for (int q = 0; q < PS_PER; ++q) {
      const uint32_t x = (uint32_t)(q * PS_THREADS + tid);
      from[q] = 0xFFFFu;
      if (x < n) {
        const uint32_t d = (gk[x] - kmin) >> sh;
        if (cur[d] - bst[d] > (uint32_t)PS_BIG) from[q] = fpos[x];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PS_PER; ++q) {
      const uint32_t x = (uint32_t)(q * PS_THREADS + tid);
      if (from[q] != 0xFFFFu) fpos[from[q]] = (uint16_t)x;
    }
    __syncthreads();
  }
  // 5. In the other buckets the rank on (key, id) gives the final position. Slot p
  //    is ranked by thread p mod 1024, so neighbouring lanes walk the same
  //    bucket in step (broadcast reads): a bucket can hold hundreds of
  //    entries (a surface facing the camera puts many Gaussians at one
  //    depth). The sorted ids and rects are then staged in LDS and written
  //    out coalesced.
  for (uint32_t p = tid; p < n; p += PS_THREADS) {
    const uint32_t kp = gk[p], ip = gi[p];
    const uint32_t d = (kp - kmin) >> sh;
    const uint32_t b0 = bst[d], b1 = cur[d];
    if (b1 - b0 > (uint32_t)PS_BIG) continue;  // sorted by the network above
    uint32_t rank = 0, i = b0;
    for (; i + 4 <= b1; i += 4) {  // four entries' loads in flight per step
      uint32_t k2[4], i2[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        k2[u] = gk[i + u];
        i2[u] = gi[i + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) rank += (k2[u] < kp || (k2[u] == kp && i2[u] < ip)) ? 1u : 0u;
    }
    for (; i < b1; ++i) {
      const uint32_t k2 = gk[i], i2 = gi[i];
      rank += (k2 < kp || (k2 == kp && i2 < ip)) ? 1u : 0u;
    }
    fpos[p] = (uint16_t)(b0 + rank);
  }
  __syncthreads();
  // each record's id moves to its final position in gk (the keys are no
  // longer needed)
#pragma unroll
  for (int q = 0; q < PS_PER; ++q) {
    if ((uint32_t)(q * PS_THREADS + tid) < n) {
      pos[q] = fpos[pos[q]];
      gk[pos[q]] = ir[q];
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < n; i += PS_THREADS) sorted_ids[roff + i] = gk[i];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PS_PER; ++q) {
    if ((uint32_t)(q * PS_THREADS + tid) < n) {
      gk[pos[q]] = (uint32_t)rr[q].x;
      gi[pos[q]] = (uint32_t)rr[q].y;
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < n; i += PS_THREADS) srect[roff + i] = make_int2((int)gk[i], (int)gi[i]);
  if (tid == 0) {
    view_total[v] = s_area;
    nsel_out[v] = n;
  }
}

// Instances of a record's rect [x0, x1] x [y0, y1] that come before tile
// (tx, ty) in row-major tile order: its full rows above ty, plus its columns
// left of tx when row ty crosses the rect.
__device__ __forceinline__ uint32_t rect_before(int x0, int y0, int x1, int y1, int tx, int ty) {
  const int rows = max(0, min(ty, y1 + 1) - y0);
  const int cols = (y0 <= ty && ty <= y1) ? max(0, min(tx, x1 + 1) - x0) : 0;
  return (uint32_t)(rows * (x1 - x0 + 1) + cols);
}

// A 256-thread workgroup per 2x2 block of tiles of one view. The 4 waves
// split the view's depth-sorted selection into 4 consecutive segments and
// keep, in order, the records whose rect meets the block, each packed with the
// 4-bit mask of the block's tiles it covers in the top bits of its id; on the
// way they sum, for each tile of the block, the instances in front of it.
// Then wave w builds the list of tile w of the block from the kept records.
constexpr int PT_THREADS = 256;
constexpr int PT_ROUND = 12;  // loads in flight per lane and array
static_assert(PS_CAP % 4 == 0 && (PS_CAP / 4) % 64 == 0, "wave segments are whole 64-record groups");

__global__ __launch_bounds__(PT_THREADS) void ptiles_kernel(ViewTab tab, const uint32_t* __restrict__ view_total,
                                                            const uint32_t* __restrict__ nsel,
                                                            const uint32_t* __restrict__ sorted_ids,
                                                            const int2* __restrict__ srect, int64_t capacity,
                                                            uint32_t* __restrict__ tile_start,
                                                            uint32_t* __restrict__ out_ids,
                                                            int64_t* __restrict__ n_inst,
                                                            int32_t* __restrict__ overflow,
                                                            int32_t* __restrict__ sticky) {
  __shared__ uint32_t s_keep[PS_CAP];
  __shared__ uint32_t s_cnt[4];
  __shared__ uint32_t s_front[4][4];  // [wave][tile of the block]
  const int v = blockIdx.y;
  const int gx = tab.gx[v], gy = tab.gy[v];
  const int nbx = (gx + 1) >> 1, nby = (gy + 1) >> 1;
  if ((int)blockIdx.x >= nbx * nby) return;  // uniform per workgroup
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
  const int X0 = bx * 2, Y0 = by * 2;
  const int64_t roff = tab.r_off[v];
  const uint32_t n = nsel[v];
  const uint64_t lmask = lanemask_lt();
  // 1. ordered compaction of the records that meet the block, per wave segment
  const uint32_t L = ((n + 3) / 4 + 63) & ~63u;  // <= PS_CAP / 4
  const uint32_t s0 = (uint32_t)w * L, s1 = min(n, s0 + L);
  uint32_t* keep = s_keep + s0;
  uint32_t kept = 0;
  uint32_t front[4] = {0u, 0u, 0u, 0u};
  for (uint32_t r0 = s0; r0 < s1; r0 += PT_ROUND * 64) {
    int2 rc[PT_ROUND];
    uint32_t idv[PT_ROUND];
#pragma unroll
    for (int u = 0; u < PT_ROUND; ++u) {
      const uint32_t i = r0 + u * 64 + lane;
      rc[u] = make_int2(1 | (1 << 16), 0);
      idv[u] = 0;
      if (i < s1) {
        rc[u] = srect[roff + i];
        idv[u] = sorted_ids[roff + i];
      }
    }
#pragma unroll
    for (int u = 0; u < PT_ROUND; ++u) {
      int x0, y0, x1, y1;
      rect_of(rc[u], x0, y0, x1, y1);
      const bool cx0 = x0 <= X0 && X0 <= x1, cx1 = x0 <= X0 + 1 && X0 + 1 <= x1;
      const bool cy0 = y0 <= Y0 && Y0 <= y1, cy1 = y0 <= Y0 + 1 && Y0 + 1 <= y1;
      const uint32_t mk = (uint32_t)(cx0 && cy0) | (uint32_t)(cx1 && cy0) << 1 | (uint32_t)(cx0 && cy1) << 2 |
                          (uint32_t)(cx1 && cy1) << 3;
      const uint64_t m = __ballot(mk != 0);
      if (mk) keep[kept + __popcll(m & lmask)] = mk << 28 | idv[u];
      kept += (uint32_t)__popcll(m);
#pragma unroll
      for (int k = 0; k < 4; ++k) front[k] += rect_before(x0, y0, x1, y1, X0 + (k & 1), Y0 + (k >> 1));
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) front[k] += (uint32_t)__shfl_xor((int)front[k], o, 64);
  }
  if (lane == 0) {
    s_cnt[w] = kept;
#pragma unroll
    for (int k = 0; k < 4; ++k) s_front[w][k] = front[k];
  }
  __syncthreads();
  // 2. wave w builds the list of tile (X0 + w % 2, Y0 + w / 2)
  const int tx = X0 + (w & 1), ty = Y0 + (w >> 1);
  if (tx >= gx || ty >= gy) return;
  const int lt = ty * gx + tx;
  const int t = tab.tile_base[v] + lt;
  const uint32_t tv = lane < tab.nv ? view_total[lane] : 0u;
  uint32_t before = lane < v ? tv : 0u, all = tv;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    before += (uint32_t)__shfl_xor((int)before, o, 64);
    all += (uint32_t)__shfl_xor((int)all, o, 64);
  }
  const uint32_t start = before + s_front[0][w] + s_front[1][w] + s_front[2][w] + s_front[3][w];
  const bool ovf = (int64_t)all > capacity;
  if (lane == 0) tile_start[t] = start;
  if (t == tab.ntiles - 1 && lane == 0) {
    tile_start[tab.ntiles] = all;
    *n_inst = all;
    *overflow = ovf ? 1 : 0;
    if (sticky && ovf) atomicOr(&sticky[0], 1);
  }
  if (ovf) return;
  uint32_t* out = out_ids + start;
  const int bit = 28 + w;
  uint32_t got = 0;
  for (int r = 0; r < 4; ++r) {
    const uint32_t c = s_cnt[r];
    const uint32_t* seg = s_keep + r * L;
    for (uint32_t i0 = 0; i0 < c; i0 += 256) {
      uint32_t e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t i = i0 + u * 64 + lane;
        e[u] = i < c ? seg[i] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool hit = (e[u] >> bit) & 1u;
        const uint64_t m = __ballot(hit);
        if (hit) out[got + __popcll(m & lmask)] = e[u] & 0x0FFFFFFFu;
        got += (uint32_t)__popcll(m);
      }
    }
  }
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ------------------------------------------------------------------ host side
struct PrefWs {
  size_t cnt, seg_key, seg_id, seg_rect, srect, vtot, nsel, nvis, bytes;
  int nb_max;
};

static PrefWs pref_layout(const ViewTab& tab) {
  PrefWs L;
  int64_t nbm = 0;
  for (int v = 0; v < tab.nv; ++v) nbm = max(nbm, (tab.npad[v] + SEL_TILE - 1) / SEL_TILE);
  L.nb_max = (int)max((int64_t)1, nbm);
  const size_t M = (size_t)tab.nrec;
  size_t o = 0;
  L.cnt = o; o += al256((size_t)tab.nv * L.nb_max * 4);
  L.seg_key = o; o += al256(M * 4);
  L.seg_id = o; o += al256(M * 4);
  L.seg_rect = o; o += al256(M * 8);
  L.srect = o; o += al256(M * 8);
  L.vtot = o; o += al256(4 * GS_MAX_VIEWS);
  L.nsel = o; o += al256(4 * GS_MAX_VIEWS);
  L.nvis = o; o += al256(4 * GS_MAX_VIEWS);
  L.bytes = o;
  return L;
}

// Raises psort's dynamic LDS limit once per context; false when the device
// cannot give a workgroup that much.
static bool prefix_lds_ok(gs_ctx* ctx) {
  if (ctx->lds_limit == 0) {
    int v = 0;
    size_t lim = 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) == hipSuccess &&
        (size_t)v >= PS_LDS + 1024) {
      if (hipFuncSetAttribute((const void*)psort_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PS_LDS) ==
          hipSuccess)
        lim = (size_t)v;
      else
        (void)hipGetLastError();
    } else {
      (void)hipGetLastError();
    }
    ctx->lds_limit = lim;
  }
  return ctx->lds_limit >= PS_LDS + 1024;
}

int64_t bin_prefix_cap() { return PS_CAP; }

size_t bin_prefix_ws_bytes(gs_ctx* ctx, const ViewTab& tab, int64_t capacity) {
  (void)ctx;
  (void)capacity;
  return pref_layout(tab).bytes;
}

gs_status launch_bin_prefix(gs_ctx* ctx, const ViewTab& tab, const gs_camera* cams, const gs_gaussians* g,
                            const gs_proj* proj, gs_bins* bins, char* ws, hipStream_t s) {
  if (!prefix_lds_ok(ctx))
    return gs_fail(ctx, GS_E_UNSUPPORTED, "prefix binning needs %zu B of LDS per workgroup", PS_LDS + 1024);
  const PrefWs L = pref_layout(tab);
  if (L.nb_max > PS_MAXBLK) return gs_fail(ctx, GS_E_UNSUPPORTED, "prefix binning: too many records per view");
  GaussSrc gsrc;
  gsrc.mean = g->mean;
  gsrc.log_scale = g->log_scale;
  gsrc.quat = g->quat;
  gsrc.opl = g->opacity_logit;
  gsrc.color = g->color;
  gsrc.mp = g->mp;
  gsrc.n = g->n;
  uint32_t* cnt = (uint32_t*)(ws + L.cnt);
  uint32_t* seg_key = (uint32_t*)(ws + L.seg_key);
  uint32_t* seg_id = (uint32_t*)(ws + L.seg_id);
  int2* seg_rect = (int2*)(ws + L.seg_rect);
  int2* srect = (int2*)(ws + L.srect);
  uint32_t* vtot = (uint32_t*)(ws + L.vtot);
  uint32_t* nsel = (uint32_t*)(ws + L.nsel);
  uint32_t* nvis = (uint32_t*)(ws + L.nvis);
  GS_LAUNCH(ctx, psel_kernel, dim3(L.nb_max, tab.nv), dim3(GS_BLOCK), 0, s, tab, proj->depth_key, proj->key_hist,
            (const int2*)proj->rect, bins->max_rank, L.nb_max, cams, gsrc, (float4*)proj->rec, seg_key, seg_id,
            seg_rect, cnt, bins->overflow, bins->incomplete, bins->truncated, nvis, proj->keys_only ? 1 : 0);
  GS_LAUNCH(ctx, psort_kernel, dim3(tab.nv), dim3(PS_THREADS), PS_LDS, s, tab, L.nb_max, cnt, seg_key, seg_id,
            seg_rect, proj->key_hist, bins->sorted_ids, srect, vtot, nsel, bins->incomplete, bins->truncated, nvis,
            bins->sticky);
  int nblk = 1;
  for (int v = 0; v < tab.nv; ++v) nblk = max(nblk, ((tab.gx[v] + 1) >> 1) * ((tab.gy[v] + 1) >> 1));
  GS_LAUNCH(ctx, ptiles_kernel, dim3(nblk, tab.nv), dim3(PT_THREADS), 0, s, tab, vtot, nsel, bins->sorted_ids, srect, bins->capacity, bins->tile_start, bins->gauss_id, bins->n_instances,
            bins->overflow, bins->sticky);
  return gs_check_launch(ctx, "bin_sort (prefix)");
}
