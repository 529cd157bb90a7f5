// Host side of the C ABI: argument validation, batch tables, workspace
// layout and kernel dispatch. Nothing here allocates device memory.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "gs_internal.h"

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

gs_status gs_fail(gs_ctx* ctx, gs_status s, const char* fmt, ...) {
  if (ctx) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

void gs_note_timer(gs_ctx* ctx, const char* name, hipEvent_t a, hipEvent_t b) {
  try {
    ctx->pending.push_back(GsTimer{name, a, b});
  } catch (...) {
    hipEventDestroy(a);
    hipEventDestroy(b);
  }
}

gs_status gs_check_launch(gs_ctx* ctx, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return gs_fail(ctx, GS_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return GS_OK;
}

extern "C" {

const char* gs_status_str(gs_status s) {
  switch (s) {
    case GS_OK: return "ok";
    case GS_E_ARG: return "invalid argument";
    case GS_E_CAPACITY: return "instance capacity exceeded";
    case GS_E_HIP: return "HIP error";
    case GS_E_UNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

gs_status gs_ctx_create(int device, gs_ctx** out) {
  if (!out) return GS_E_ARG;
  *out = nullptr;
  gs_ctx* c = new (std::nothrow) gs_ctx;
  if (!c) return GS_E_HIP;
  c->device = device;
  c->render_batch = 128;
  c->bwd_batch = 64;
  c->bin_chunk = 1024;
  c->timing = 0;
  c->tile_order = 1;
  c->bwd_copies = 8;
  c->wave_cull = 1;
  c->n_cu = 0;
  c->proj_resident = 0;
  c->lds_limit = 0;
  c->no_alloc = 0;
  c->exact_keys = 0;
  c->err[0] = 0;
  *out = c;
  return GS_OK;
}

gs_status gs_ctx_destroy(gs_ctx* ctx) {
  if (ctx) {
    for (auto& t : ctx->pending) {
      hipEventDestroy(t.a);
      hipEventDestroy(t.b);
    }
  }
  delete ctx;
  return GS_OK;
}

gs_status gs_ctx_kernel_times(gs_ctx* ctx, char* buf, size_t len) {
  if (!ctx || !buf || len == 0) return GS_E_ARG;
  struct Acc {
    const char* name;
    long n;
    double ms;
  };
  // at most one row per kernel name: a fixed table, no allocation
  constexpr size_t kMaxNames = 64;
  Acc acc_tab[kMaxNames];
  size_t n_acc = 0;
  gs_status st = GS_OK;
  for (auto& t : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess)
      st = gs_fail(ctx, GS_E_HIP, "reading kernel timing events failed");
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
    size_t i = 0;
    while (i < n_acc && strcmp(acc_tab[i].name, t.name) != 0) ++i;
    if (i == n_acc) {
      if (n_acc == kMaxNames) continue;
      acc_tab[n_acc++] = Acc{t.name, 0, 0.0};
    }
    acc_tab[i].n += 1;
    acc_tab[i].ms += ms;
  }
  ctx->pending.clear();
  size_t o = 0;
  buf[0] = 0;
  for (size_t i = 0; i < n_acc; ++i) {
    const Acc& a = acc_tab[i];
    const int w = snprintf(buf + o, len - o, "%s %ld %.6f\n", a.name, a.n, a.ms);
    if (w < 0 || (size_t)w >= len - o) break;
    o += (size_t)w;
  }
  return st;
}

const char* gs_last_error(const gs_ctx* ctx) { return ctx ? ctx->err : "null context"; }

gs_status gs_ctx_set_param(gs_ctx* ctx, const char* name, int64_t value) {
  if (!ctx || !name) return GS_E_ARG;
  if (!strcmp(name, "render_batch")) {
    if (value != 64 && value != 128 && value != 256) return gs_fail(ctx, GS_E_ARG, "render_batch: 64|128|256");
    ctx->render_batch = (int)value;
  } else if (!strcmp(name, "bwd_batch")) {
    if (value != 32 && value != 64 && value != 128) return gs_fail(ctx, GS_E_ARG, "bwd_batch: 32|64|128");
    ctx->bwd_batch = (int)value;
  } else if (!strcmp(name, "timing")) {
    ctx->timing = value ? 1 : 0;
  } else if (!strcmp(name, "bwd_copies")) {
    if (value != 1 && value != 2 && value != 4 && value != 8) return gs_fail(ctx, GS_E_ARG, "bwd_copies: 1|2|4|8");
    ctx->bwd_copies = (int)value;
  } else if (!strcmp(name, "wave_cull")) {
    if (value != 0 && value != 1) return gs_fail(ctx, GS_E_ARG, "wave_cull: 0|1");
    ctx->wave_cull = (int)value;
  } else if (!strcmp(name, "tile_order")) {
    if (value != 0 && value != 1) return gs_fail(ctx, GS_E_ARG, "tile_order: 0|1");
    ctx->tile_order = (int)value;
  } else if (!strcmp(name, "exact_keys")) {
    if (value != 0 && value != 1) return gs_fail(ctx, GS_E_ARG, "exact_keys: 0|1");
    ctx->exact_keys = (int)value;
  } else if (!strcmp(name, "bin_chunk")) {
    if (value != 256 && value != 512 && value != 1024 && value != 2048)
      return gs_fail(ctx, GS_E_ARG, "bin_chunk: 256|512|1024|2048");
    ctx->bin_chunk = (int)value;
  } else {
    return gs_fail(ctx, GS_E_ARG, "unknown parameter %s", name);
  }
  return GS_OK;
}

gs_status gs_ctx_get_param(const gs_ctx* ctx, const char* name, int64_t* value) {
  if (!ctx || !name || !value) return GS_E_ARG;
  if (!strcmp(name, "render_batch")) *value = ctx->render_batch;
  else if (!strcmp(name, "bwd_batch")) *value = ctx->bwd_batch;
  else if (!strcmp(name, "bin_chunk")) *value = ctx->bin_chunk;
  else if (!strcmp(name, "timing")) *value = ctx->timing;
  else if (!strcmp(name, "tile_order")) *value = ctx->tile_order;
  else if (!strcmp(name, "wave_cull")) *value = ctx->wave_cull;
  else if (!strcmp(name, "bwd_copies")) *value = ctx->bwd_copies;
  else if (!strcmp(name, "exact_keys")) *value = ctx->exact_keys;
  else if (!strcmp(name, "n_cu")) *value = ctx->n_cu;
  else if (!strcmp(name, "lds_limit")) *value = (int64_t)ctx->lds_limit;
  else if (!strcmp(name, "prefix_cap")) *value = bin_prefix_cap();
  else return GS_E_ARG;
  return GS_OK;
}

}  // extern "C"

// Builds the per-batch table; validates the views.
static gs_status make_tab(gs_ctx* ctx, const gs_views* vw, ViewTab& tab) {
  std::memset(&tab, 0, sizeof(tab));
  if (!vw) return gs_fail(ctx, GS_E_ARG, "views is NULL");
  const int64_t n_total = vw->n_gaussians;
  if (vw->n_views < 1 || vw->n_views > GS_MAX_VIEWS)
    return gs_fail(ctx, GS_E_ARG, "n_views must be in [1, %d]", GS_MAX_VIEWS);
  if (!vw->cams_host || !vw->cams_dev) return gs_fail(ctx, GS_E_ARG, "cameras are NULL");
  const int S = vw->n_scenes < 1 ? 1 : vw->n_scenes;
  if (n_total < 0) return gs_fail(ctx, GS_E_ARG, "n < 0");
  if (!vw->scene_begin && S != 1) return gs_fail(ctx, GS_E_ARG, "scene_begin required for n_scenes > 1");
  if (vw->scene_begin) {
    if (vw->scene_begin[0] != 0 || vw->scene_begin[S] != n_total)
      return gs_fail(ctx, GS_E_ARG, "scene_begin must run from 0 to n");
    for (int s = 0; s < S; ++s)
      if (vw->scene_begin[s + 1] < vw->scene_begin[s]) return gs_fail(ctx, GS_E_ARG, "scene_begin not monotone");
  }
  tab.nv = vw->n_views;
  tab.ng = n_total;
  int64_t roff = 0, poff = 0;
  int32_t tb = 0;
  for (int v = 0; v < tab.nv; ++v) {
    const int s = vw->view_scene ? vw->view_scene[v] : 0;
    if (s < 0 || s >= S) return gs_fail(ctx, GS_E_ARG, "view %d: scene %d out of range", v, s);
    const gs_camera& c = vw->cams_host[v];
    if (c.width <= 0 || c.height <= 0) return gs_fail(ctx, GS_E_ARG, "view %d: empty image", v);
    const int gx = (c.width + GS_TILE - 1) / GS_TILE, gy = (c.height + GS_TILE - 1) / GS_TILE;
    if ((gx + 1) * (gy + 1) > 4096) return gs_fail(ctx, GS_E_UNSUPPORTED, "view %d: image too large", v);
    const int64_t b = vw->scene_begin ? vw->scene_begin[s] : 0;
    const int64_t e = vw->scene_begin ? vw->scene_begin[s + 1] : n_total;
    tab.W[v] = c.width;
    tab.H[v] = c.height;
    tab.gx[v] = gx;
    tab.gy[v] = gy;
    tab.scene[v] = s;
    tab.tile_base[v] = tb;
    tab.n[v] = e - b;
    tab.npad[v] = (e - b + 63) / 64 * 64;
    tab.g_off[v] = b;
    tab.r_off[v] = roff;
    tab.px_off[v] = poff;
    roff += tab.npad[v];
    poff += (int64_t)c.width * c.height;
    tb += gx * gy;
  }
  tab.tile_base[tab.nv] = tb;
  tab.ntiles = tb;
  tab.nrec = roff;
  tab.npix = poff;
  if (roff >= (int64_t)1 << 32) return gs_fail(ctx, GS_E_UNSUPPORTED, "more than 2^32 records");
  return GS_OK;
}

struct BwdWs {
  size_t g2d, flag, list, counters, pose, bytes;
};
static BwdWs bwd_ws_layout(gs_ctx* ctx, const ViewTab& tab) {
  BwdWs L;
  size_t o = 0;
  L.g2d = o; o += al256((size_t)tab.nrec * 10 * 4 * (size_t)ctx->bwd_copies);
  L.flag = o; o += al256((size_t)tab.ng * 4);
  L.list = o; o += al256((size_t)tab.ng * 4);
  L.counters = o; o += 256;
  L.pose = o; o += al256((size_t)kChainBlocks * tab.nv * 6 * 4);
  L.bytes = o;
  return L;
}

#define GS_TRY(x)                 \
  do {                            \
    const gs_status st_ = (x);    \
    if (st_ != GS_OK) return st_; \
  } while (0)

extern "C" {

int64_t gs_rec_offset(const gs_views* views, int32_t view) {
  ViewTab tab;
  if (make_tab(nullptr, views, tab) != GS_OK || view < 0 || view >= tab.nv) return -1;
  return tab.r_off[view];
}

int64_t gs_rec_count(const gs_views* views) {
  ViewTab tab;
  if (make_tab(nullptr, views, tab) != GS_OK) return -1;
  return tab.nrec;
}

int64_t gs_tile_count(const gs_views* views) {
  ViewTab tab;
  if (make_tab(nullptr, views, tab) != GS_OK) return -1;
  return tab.ntiles;
}

int64_t gs_pixel_count(const gs_views* views) {
  if (!views || !views->cams_host || views->n_views < 1) return -1;
  int64_t p = 0;
  for (int v = 0; v < views->n_views; ++v) p += (int64_t)views->cams_host[v].width * views->cams_host[v].height;
  return p;
}

// Float64 partials of gs_loss (one per 256 pixels of each view) or of
// gs_render_fwd_loss (one per tile), whichever is larger.
static size_t loss_ws_bytes(const ViewTab& tab) {
  const size_t a = (size_t)tab.nv * loss_blocks(tab), b = (size_t)tab.ntiles;
  return al256((a > b ? a : b) * 8 + 8);
}

gs_status gs_workspace_size(gs_ctx* ctx, const gs_views* views, int32_t op, int64_t capacity, size_t* bytes) {
  if (!ctx || !bytes) return GS_E_ARG;
  if (op == GS_OP_COMPACT || op == GS_OP_MP_REG) {
    if (capacity < 0) return gs_fail(ctx, GS_E_ARG, "n < 0");
    *bytes = op == GS_OP_COMPACT ? compact_ws_bytes(capacity) : mp_reg_ws_bytes(capacity);
    return GS_OK;
  }
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  switch (op) {
    case GS_OP_BIN_SORT: {
      if (capacity < 0) return gs_fail(ctx, GS_E_ARG, "capacity < 0");
      BinTab bt;
      bin_tab_fill(tab, ctx->bin_chunk, 0, bt);
      // the smallest chunk gives the largest count matrix
      BinTab bt2;
      bin_tab_fill(tab, 256, 0, bt2);
      size_t a = bin_ws_layout(tab, bt).bytes, b = bin_ws_layout(tab, bt2).bytes;
      a = a > b ? a : b;
      b = bin_prefix_ws_bytes(ctx, tab, capacity);
      *bytes = a > b ? a : b;
      return GS_OK;
    }
    case GS_OP_RENDER_BWD: *bytes = bwd_ws_layout(ctx, tab).bytes; return GS_OK;
    case GS_OP_LOSS: *bytes = loss_ws_bytes(tab); return GS_OK;
    case GS_OP_MP_UPDATE:
      if (tab.nv != 1) return gs_fail(ctx, GS_E_ARG, "mp_update takes one view");
      *bytes = mp_ws_bytes(tab, tab.npix);
      return GS_OK;
    case GS_OP_MLP_TRAIN: *bytes = mlp_ws_bytes(tab.npix); return GS_OK;
    case GS_OP_EDGE_WARP:
      if (capacity < 0 || capacity > GS_MAX_VIEWS) return gs_fail(ctx, GS_E_ARG, "n_pairs must be in [0, %d]", GS_MAX_VIEWS);
      *bytes = edge_warp_ws_bytes(tab, (int32_t)capacity);
      return GS_OK;
    default: return gs_fail(ctx, GS_E_ARG, "unknown op %d", op);
  }
}

gs_status gs_project(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, gs_proj* proj, void* stream) {
  if (!ctx || !g || !proj) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (g->n != tab.ng) return gs_fail(ctx, GS_E_ARG, "gaussians.n != views.n_gaussians");
  if (g->n > 0 && (!g->mean || !g->log_scale || !g->quat || !g->opacity_logit || !g->color || !g->mp))
    return gs_fail(ctx, GS_E_ARG, "gaussian arrays are NULL");
  if (tab.nrec > 0 && (!proj->rec || !proj->rect || !proj->depth_key))
    return gs_fail(ctx, GS_E_ARG, "proj.rec/rect/depth_key NULL");
  if (proj->m < tab.nrec) return gs_fail(ctx, GS_E_ARG, "proj.m %lld < %lld records", (long long)proj->m,
                                         (long long)tab.nrec);
  return launch_project(ctx, tab, views->cams_dev, g, proj, (hipStream_t)stream);
}

gs_status gs_bin_sort(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, gs_proj* proj, gs_bins* bins,
                      void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !proj || !bins) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (!bins->gauss_id || !bins->tile_start || (tab.nrec > 0 && !bins->sorted_ids) || !bins->n_instances ||
      !bins->overflow || !bins->incomplete)
    return gs_fail(ctx, GS_E_ARG, "bins arrays NULL");
  if (bins->capacity < 0 || bins->capacity > ((int64_t)1 << 32)) return gs_fail(ctx, GS_E_ARG, "bad capacity");
  if (bins->max_rank > 0 && !bins->truncated) return gs_fail(ctx, GS_E_ARG, "bins.truncated NULL with max_rank > 0");
  if (bins->max_rank > 0 && proj->key_hist) {
    const size_t need = bin_prefix_ws_bytes(ctx, tab, bins->capacity);
    if (!ws || ws_bytes < need) return gs_fail(ctx, GS_E_ARG, "bin_sort workspace %zu < %zu bytes", ws_bytes, need);
    if (!g || g->n != tab.ng || (tab.nrec > 0 && !proj->rec))
      return gs_fail(ctx, GS_E_ARG, "prefix binning needs the gaussians and proj.rec");
    return launch_bin_prefix(ctx, tab, views->cams_dev, g, proj, bins, (char*)ws, (hipStream_t)stream);
  }
  // the full lists read the rect and record of every Gaussian, which
  // gs_project writes only when key_hist is NULL
  if (proj->key_hist)
    return gs_fail(ctx, GS_E_ARG,
                   "full-list binning (max_rank <= 0) needs a projection run with proj.key_hist NULL: with it set, "
                   "gs_project writes no compositing records%s",
                   proj->keys_only ? " and no tile rects" : "");
  BinTab bt;
  bin_tab_fill(tab, ctx->bin_chunk, bins->max_rank, bt);
  const BinWs L = bin_ws_layout(tab, bt);
  if (!ws || ws_bytes < L.bytes)
    return gs_fail(ctx, GS_E_ARG, "bin_sort workspace %zu < %zu bytes", ws_bytes, L.bytes);
  return launch_bin_sort(ctx, tab, bt, proj, bins, (char*)ws, (hipStream_t)stream);
}

gs_status gs_render_fwd(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                        const gs_bins* bins, const float* bg, gs_image* img, void* stream) {
  if (!ctx || !g || !proj || !bins || !bg || !img) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (!img->color || !img->depth || !img->mp || !img->T || !img->n_last) return gs_fail(ctx, GS_E_ARG, "image NULL");
  if (g->n != tab.ng) return gs_fail(ctx, GS_E_ARG, "gaussians.n != views.n_gaussians");
  if (bins->max_rank > 0 && !bins->truncated) return gs_fail(ctx, GS_E_ARG, "bins.truncated NULL with max_rank > 0");
  return launch_render_fwd(ctx, tab, proj, bins, bg, img, (hipStream_t)stream);
}

gs_status gs_loss(gs_ctx* ctx, const gs_views* views, const gs_image* img, const gs_target* tgt,
                  const gs_loss_params* lp, float* loss, gs_pixel_grads* pg, void* ws, size_t ws_bytes,
                  void* stream) {
  if (!ctx || !img || !tgt || !lp || !loss || !pg) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (!pg->dcolor || !pg->ddepth) return gs_fail(ctx, GS_E_ARG, "pixel grads NULL");
  if (lp->weight_mode != 0 && lp->weight_mode != 1) return gs_fail(ctx, GS_E_ARG, "weight_mode 0|1");
  const size_t need = loss_ws_bytes(tab);
  if (!ws || ws_bytes < need) return gs_fail(ctx, GS_E_ARG, "loss workspace %zu < %zu", ws_bytes, need);
  return launch_loss(ctx, tab, img, tgt, lp, loss, pg, (double*)ws, (hipStream_t)stream);
}

gs_status gs_render_fwd_loss(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                             const gs_bins* bins, const float* bg, gs_image* img, const gs_target* tgt,
                             const gs_loss_params* lp, float* loss, gs_pixel_grads* pg, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!ctx || !g || !proj || !bins || !bg || !img || !tgt || !lp || !loss || !pg)
    return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (!img->color || !img->depth || !img->mp || !img->T || !img->n_last) return gs_fail(ctx, GS_E_ARG, "image NULL");
  if (g->n != tab.ng) return gs_fail(ctx, GS_E_ARG, "gaussians.n != views.n_gaussians");
  if (!tgt->color || !tgt->depth) return gs_fail(ctx, GS_E_ARG, "target NULL");
  if (!pg->dcolor || !pg->ddepth) return gs_fail(ctx, GS_E_ARG, "pixel grads NULL");
  if (lp->weight_mode != 0 && lp->weight_mode != 1) return gs_fail(ctx, GS_E_ARG, "weight_mode 0|1");
  const size_t need = loss_ws_bytes(tab);
  if (!ws || ws_bytes < need) return gs_fail(ctx, GS_E_ARG, "loss workspace %zu < %zu", ws_bytes, need);
  if (bins->max_rank > 0 && !bins->truncated) return gs_fail(ctx, GS_E_ARG, "bins.truncated NULL with max_rank > 0");
  const LossArgs la = loss_args(tgt, lp, pg, (double*)ws, loss);
  return launch_render_fwd(ctx, tab, proj, bins, bg, img, (hipStream_t)stream, &la);
}

}  // extern "C"

// Scratch of the allocation-free forward + loss: one float64 loss partial per
// tile. Every call overwrites the partial of each tile of its batch before
// the per-view sums read them, so nothing needs clearing between calls.
static constexpr int64_t kStaticLossTiles = 32768;  // 256 KiB
static __device__ __align__(256) double scratch[kStaticLossTiles];

// Device address of `scratch` on each device, resolved on the first call
// made with that device current (hipGetSymbolAddress). The array's host-side
// name is not a device address and is never handed to a kernel.
static constexpr int kMaxDevices = 64;
static double* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static gs_status static_scratch(gs_ctx* ctx, double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return gs_fail(ctx, GS_E_HIP, "no current device (or device index >= %d)", kMaxDevices);
  try {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return gs_fail(ctx, GS_E_HIP, "resolving the static loss scratch on device %d: %s", dev,
                       hipGetErrorString(e));
      g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
  } catch (...) {
    return gs_fail(ctx, GS_E_HIP, "locking the static scratch table failed");
  }
  return GS_OK;
}

extern "C" {

gs_status gs_render_fwd_loss_static(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                                    const gs_bins* bins, const float* bg, gs_image* img, const gs_target* tgt,
                                    const gs_loss_params* lp, float* loss, gs_pixel_grads* pg, void* stream) {
  if (!ctx || !g || !proj || !bins || !bg || !img || !tgt || !lp || !loss || !pg)
    return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (!img->color || !img->depth || !img->mp || !img->T || !img->n_last) return gs_fail(ctx, GS_E_ARG, "image NULL");
  if (g->n != tab.ng) return gs_fail(ctx, GS_E_ARG, "gaussians.n != views.n_gaussians");
  if (!tgt->color || !tgt->depth) return gs_fail(ctx, GS_E_ARG, "target NULL");
  if (!pg->dcolor || !pg->ddepth) return gs_fail(ctx, GS_E_ARG, "pixel grads NULL");
  if (lp->weight_mode != 0 && lp->weight_mode != 1) return gs_fail(ctx, GS_E_ARG, "weight_mode 0|1");
  if (tab.ntiles > kStaticLossTiles)
    return gs_fail(ctx, GS_E_UNSUPPORTED, "the batch has %lld tiles; gs_render_fwd_loss_static holds at most %lld",
                   (long long)tab.ntiles, (long long)kStaticLossTiles);
  double* part = nullptr;
  GS_TRY(static_scratch(ctx, &part));
  if (bins->max_rank > 0 && !bins->truncated) return gs_fail(ctx, GS_E_ARG, "bins.truncated NULL with max_rank > 0");
  const LossArgs la = loss_args(tgt, lp, pg, part, loss);
  ctx->no_alloc = 1;
  const gs_status st = launch_render_fwd(ctx, tab, proj, bins, bg, img, (hipStream_t)stream, &la);
  ctx->no_alloc = 0;
  return st;
}

gs_status gs_render_bwd(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                        const gs_bins* bins, const gs_image* img, const gs_pixel_grads* pg, const float* bg,
                        gs_grads* gr, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !g || !proj || !bins || !img || !pg || !bg || !gr) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (g->n != tab.ng) return gs_fail(ctx, GS_E_ARG, "gaussians.n != views.n_gaussians");
  if (!gr->pose_only && tab.ng > 0 && (!gr->mean || !gr->log_scale || !gr->quat || !gr->opacity_logit || !gr->color))
    return gs_fail(ctx, GS_E_ARG, "gradient arrays NULL");
  const BwdWs L = bwd_ws_layout(ctx, tab);
  if (!ws || ws_bytes < L.bytes) return gs_fail(ctx, GS_E_ARG, "render_bwd workspace %zu < %zu", ws_bytes, L.bytes);
  char* w = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  TouchArgs touch;
  touch.flag = (uint32_t*)(w + L.flag);
  touch.list = (uint32_t*)(w + L.list);
  touch.count = (uint32_t*)(w + L.counters);
  touch.ticket = touch.count + 1;
  GS_TRY(launch_render_bwd_tiles(ctx, tab, proj, bins, img, pg, bg, (float*)(w + L.g2d), touch, gr, s));
  return launch_bwd_project(ctx, tab, views->cams_dev, g, (float*)(w + L.g2d), touch, (float*)(w + L.pose), gr, s);
}

gs_status gs_bins_check(gs_ctx* ctx, const gs_bins* bins, int64_t* required, int32_t* incomplete, void* stream) {
  if (!ctx || !bins || !required) return GS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  int64_t n = 0;
  int32_t of = 0, inc = 0;
  if (hipStreamSynchronize(s) != hipSuccess) return gs_fail(ctx, GS_E_HIP, "stream sync failed");
  if (hipMemcpy(&n, bins->n_instances, 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&of, bins->overflow, 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&inc, bins->incomplete, 4, hipMemcpyDeviceToHost) != hipSuccess)
    return gs_fail(ctx, GS_E_HIP, "reading bin counters failed");
  *required = n;
  if (incomplete) *incomplete = inc;
  return of ? GS_E_CAPACITY : GS_OK;
}

gs_status gs_mp_update(gs_ctx* ctx, const gs_views* views, const gs_proj* proj, const gs_image* img,
                       const gs_target* tgt, const gs_mp_frame* fr, const gs_mp_params* mp_params, float* mp,
                       gs_mp_out* out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !proj || !img || !tgt || !fr || !mp_params || !mp || !out) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (tab.nv != 1) return gs_fail(ctx, GS_E_ARG, "gs_mp_update takes exactly one view");
  if (!proj->mean2d) return gs_fail(ctx, GS_E_ARG, "proj.mean2d is required");
  if (fr->n_inst < 0 || fr->n_inst > 15) return gs_fail(ctx, GS_E_UNSUPPORTED, "n_inst must be in [0, 15]");
  if (!fr->instance_id || !fr->inst_prior || !fr->inst_conf) return gs_fail(ctx, GS_E_ARG, "frame arrays NULL");
  if (!(mp_params->radius_px >= 0.f && mp_params->radius_px <= 4.f))
    return gs_fail(ctx, GS_E_UNSUPPORTED, "radius_px must be in [0, 4]");
  if (!out->U_tilde || !out->alpha || !out->dynamic || !out->prune || !out->stats)
    return gs_fail(ctx, GS_E_ARG, "mp outputs NULL");
  const size_t need = mp_ws_bytes(tab, tab.npix);
  if (!ws || ws_bytes < need) return gs_fail(ctx, GS_E_ARG, "mp_update workspace %zu < %zu", ws_bytes, need);
  return launch_mp_update(ctx, tab, proj, img, tgt, fr, mp_params, mp, out, (char*)ws, (hipStream_t)stream);
}

gs_status gs_mp_regularizer(gs_ctx* ctx, int64_t n, const float* mean, const float* mean_prev, const float* mp,
                            const float* T, float lambda, float* loss, float* dmean, void* ws, size_t ws_bytes,
                            void* stream) {
  if (!ctx || n < 0 || !loss) return gs_fail(ctx, GS_E_ARG, "bad argument");
  if (n > 0 && (!mean || !mean_prev || !mp || !dmean)) return gs_fail(ctx, GS_E_ARG, "arrays are NULL");
  const size_t need = mp_reg_ws_bytes(n);
  if (!ws || ws_bytes < need) return gs_fail(ctx, GS_E_ARG, "mp_regularizer workspace %zu < %zu", ws_bytes, need);
  return launch_mp_reg(ctx, n, mean, mean_prev, mp, T, lambda, loss, dmean, (double*)ws, (hipStream_t)stream);
}

gs_status gs_edge_warp(gs_ctx* ctx, const gs_views* views, const gs_image* img, const gs_target* tgt,
                       const gs_edge_pair* pairs, int32_t n_pairs, const gs_edge_params* ep, float* loss,
                       float* ddepth, float* dpose, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !img || !tgt || !ep || !loss || !ddepth) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (!img->depth || !img->mp || !img->T || !tgt->depth) return gs_fail(ctx, GS_E_ARG, "image or target NULL");
  if (n_pairs < 0 || n_pairs > GS_MAX_VIEWS || (n_pairs > 0 && !pairs))
    return gs_fail(ctx, GS_E_ARG, "n_pairs must be in [0, %d]", GS_MAX_VIEWS);
  for (int k = 0; k < n_pairs; ++k)
    if (pairs[k].i < 0 || pairs[k].i >= tab.nv || pairs[k].j < 0 || pairs[k].j >= tab.nv || pairs[k].i == pairs[k].j)
      return gs_fail(ctx, GS_E_ARG, "pair %d: views (%d, %d) invalid", k, pairs[k].i, pairs[k].j);
  if (!(ep->delta > 0.f) || !(ep->edge_thresh >= 0.f)) return gs_fail(ctx, GS_E_ARG, "delta > 0, edge_thresh >= 0");
  const size_t need = edge_warp_ws_bytes(tab, n_pairs);
  if (n_pairs > 0 && (!ws || ws_bytes < need))
    return gs_fail(ctx, GS_E_ARG, "edge_warp workspace %zu < %zu", ws_bytes, need);
  return launch_edge_warp(ctx, tab, views->cams_dev, img, tgt, pairs, n_pairs, ep, loss, ddepth, dpose, (double*)ws,
                          (hipStream_t)stream);
}

gs_status gs_epipolar_verify(gs_ctx* ctx, const gs_views* views, int32_t view1, int32_t view2, const float* p1,
                             const float* p2, int64_t m, const int32_t* ids, const int64_t* seg, int64_t k,
                             const gs_epi_params* prm, float* d, float* dbar, uint8_t* state, float* mp,
                             void* stream) {
  if (!ctx || !prm || m < 0 || k < 0) return gs_fail(ctx, GS_E_ARG, "bad argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (view1 < 0 || view1 >= tab.nv || view2 < 0 || view2 >= tab.nv || view1 == view2)
    return gs_fail(ctx, GS_E_ARG, "views (%d, %d) invalid", view1, view2);
  if (m > 0 && (!p1 || !p2 || !d)) return gs_fail(ctx, GS_E_ARG, "match arrays are NULL");
  if (k > 0 && (!ids || !seg || !dbar || !state || (tab.ng > 0 && !mp)))
    return gs_fail(ctx, GS_E_ARG, "candidate arrays are NULL");
  if (!(prm->eps >= 0.f) || prm->tau != prm->tau) return gs_fail(ctx, GS_E_ARG, "eps >= 0 and tau not NaN");
  return launch_epipolar(ctx, views->cams_dev, view1, view2, p1, p2, m, ids, seg, k, tab.ng, prm->eps, prm->tau,
                         prm->mp_restore, d, dbar, state, mp, (hipStream_t)stream);
}

gs_status gs_sched_decide(const gs_sched_params* p, gs_sched_state* st, float U_bar, const float* dbar,
                          const uint8_t* epi_state, int64_t k, int32_t* refresh) {
  if (!p || !st || !refresh || k < 0 || (k > 0 && (!dbar || !epi_state))) return GS_E_ARG;
  if (!(p->w_u >= 0.f) || !(p->w_r >= 0.f) || !(fabs((double)p->w_u + p->w_r - 1.0) <= 1e-6) || !(p->e_ref > 0.f) ||
      p->n_max < 1)
    return GS_E_ARG;
  // e_bar: mean of the finite medians of the candidates MP labels static,
  // summed in candidate order in double
  double sum = 0.0;
  int64_t cnt = 0;
  for (int64_t i = 0; i < k; ++i)
    if (epi_state[i] == GS_EPI_NOT_SUPPRESSED && std::isfinite(dbar[i])) {
      sum += dbar[i];
      ++cnt;
    }
  const float e_bar = cnt ? (float)(sum / (double)cnt) : 0.f;
  float R = e_bar / p->e_ref;
  R = R < 0.f ? 0.f : (R > 1.f ? 1.f : R);
  const float U = U_bar != U_bar ? 0.f : U_bar;
  const float S = p->w_u * U + p->w_r * R;
  const int32_t dt = st->dt < 0 ? 0 : st->dt;
  const bool go = S > p->theta || dt >= p->n_max;
  st->S = S;
  st->R = R;
  st->e_bar = e_bar;
  if (go) {
    st->dt = 1;
    st->n_refresh += 1;
  } else {
    st->dt = dt + 1;
  }
  *refresh = go ? 1 : 0;
  return GS_OK;
}

gs_status gs_compact(gs_ctx* ctx, const uint8_t* drop, int64_t n, int32_t n_planes, const float* const* src,
                     float* const* dst, const int64_t* seg_begin, int32_t n_seg, int64_t* seg_out, int64_t* n_out,
                     void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !n_out || n < 0 || n_planes < 0) return gs_fail(ctx, GS_E_ARG, "bad argument");
  if (n > 0 && !drop) return gs_fail(ctx, GS_E_ARG, "drop is NULL");
  if (n_planes > GS_COMPACT_MAX_PLANES)
    return gs_fail(ctx, GS_E_UNSUPPORTED, "at most %d planes per call", GS_COMPACT_MAX_PLANES);
  if (n_planes > 0 && (!src || !dst)) return gs_fail(ctx, GS_E_ARG, "plane tables are NULL");
  for (int p = 0; p < n_planes; ++p) {
    if (n > 0 && (!src[p] || !dst[p])) return gs_fail(ctx, GS_E_ARG, "plane %d is NULL", p);
    if (n > 0 && (const char*)src[p] < (const char*)(dst[p] + n) && (const char*)dst[p] < (const char*)(src[p] + n))
      return gs_fail(ctx, GS_E_ARG, "plane %d: source and destination overlap", p);
  }
  if (seg_out) {
    if (n_seg < 1 || n_seg > GS_COMPACT_MAX_SEGS)
      return n_seg < 1 ? gs_fail(ctx, GS_E_ARG, "n_seg must be >= 1")
                       : gs_fail(ctx, GS_E_UNSUPPORTED, "at most %d segments", GS_COMPACT_MAX_SEGS);
    if (!seg_begin || seg_begin[0] != 0 || seg_begin[n_seg] != n)
      return gs_fail(ctx, GS_E_ARG, "seg_begin must run from 0 to n");
    for (int i = 0; i < n_seg; ++i)
      if (seg_begin[i + 1] < seg_begin[i]) return gs_fail(ctx, GS_E_ARG, "seg_begin not monotone");
  }
  const size_t need = compact_ws_bytes(n);
  if (!ws || ws_bytes < need) return gs_fail(ctx, GS_E_ARG, "compact workspace %zu < %zu", ws_bytes, need);
  return launch_compact(ctx, drop, n, n_planes, src, dst, seg_begin, n_seg, seg_out, n_out, (char*)ws,
                        (hipStream_t)stream);
}

gs_status gs_mlp_features(gs_ctx* ctx, const gs_views* views, const gs_image* img, const gs_target* tgt,
                          const gs_mp_frame* fr, float* x, void* stream) {
  if (!ctx || !img || !tgt || !fr || !x) return gs_fail(ctx, GS_E_ARG, "null argument");
  ViewTab tab;
  GS_TRY(make_tab(ctx, views, tab));
  if (!fr->instance_id || !fr->inst_prior) return gs_fail(ctx, GS_E_ARG, "frame arrays NULL");
  return launch_mlp_features(ctx, tab, img, tgt, fr, x, (hipStream_t)stream);
}

gs_status gs_mlp_sync(gs_ctx* ctx, gs_mlp* mlp, void* stream) {
  if (!ctx || !mlp || !mlp->master || !mlp->w_bf16) return gs_fail(ctx, GS_E_ARG, "null argument");
  return launch_mlp_sync(ctx, mlp, (hipStream_t)stream);
}

gs_status gs_mlp_fwd(gs_ctx* ctx, const gs_mlp* mlp, const float* x, float* y, int64_t P, void* stream) {
  if (!ctx || !mlp || !mlp->master || !mlp->w_bf16 || !x || !y || P < 0) return gs_fail(ctx, GS_E_ARG, "bad argument");
  return launch_mlp_fwd(ctx, mlp, x, y, P, (hipStream_t)stream);
}

gs_status gs_mlp_train_step(gs_ctx* ctx, gs_mlp* mlp, const float* x, const float* label, int64_t P, float lr,
                            int32_t step, float* loss, float* grad, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !mlp || !mlp->master || !mlp->w_bf16 || !mlp->adam_m || !mlp->adam_v || !x || !label || !loss ||
      P <= 0 || step < 1)
    return gs_fail(ctx, GS_E_ARG, "bad argument");
  const size_t need = mlp_ws_bytes(P);
  if (!ws || ws_bytes < need) return gs_fail(ctx, GS_E_ARG, "mlp workspace %zu < %zu", ws_bytes, need);
  return launch_mlp_train(ctx, mlp, x, label, P, lr, step, loss, grad, (char*)ws, (hipStream_t)stream);
}

}  // extern "C"
