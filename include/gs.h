/*
 * gs.h - C ABI of the MI355X (gfx950) MP-weighted Gaussian-splatting library.
 *
 * The method (DAGS-SLAM, arXiv 2602.21644) renders colour and depth from a
 * Gaussian map and a camera pose, weights the photometric and depth L1 losses
 * by a per-pixel static weight built from per-Gaussian motion probabilities
 * (Sec. IV-D, Eq. (20)-(22), (27)), optimises Gaussians and poses jointly
 * (Sec. IV-D, "Overall objective"), and keeps the motion probabilities as a
 * temporally updated state (Sec. IV-A/B, Eq. (1)-(13), (17)).
 *
 * The calls, in the order one optimisation iteration uses them:
 *   gs_project    -> gs_bin_sort -> gs_render_fwd -> gs_loss -> gs_render_bwd
 * (gs_render_fwd_loss does the middle two in one pass) and once per frame
 * gs_mp_update. The learned MP surrogate (not in the paper)
 * adds gs_mlp_features / gs_mlp_fwd / gs_mlp_train_step.
 *
 * Conventions shared by every call
 *  - Pointers are DEVICE pointers unless marked [host]. The caller owns every
 *    buffer; the library never allocates, frees or retains caller memory in a
 *    hot call. Scratch memory is the caller's `ws` of gs_workspace_size bytes.
 *  - Every hot call only enqueues work on `stream` (a hipStream_t passed as
 *    void*) and does not synchronise, so it can be captured in a hip graph.
 *    gs_bins_check is the only call that synchronises.
 *  - Return codes: GS_OK, or GS_E_ARG (bad argument, checked on the host
 *    before anything is enqueued), GS_E_UNSUPPORTED (a size beyond the
 *    library's limits), GS_E_HIP (a launch failed; text in gs_last_error).
 *    Device-side capacity overflow is reported by the overflow flag of
 *    gs_bins (kernels after it early-exit) and by gs_bins_check.
 *  - Layouts: planar float32 structure-of-arrays. A Gaussian attribute with c
 *    components is stored as c planes of length n: element (c, k) at c*n + k.
 *    Images are planar per channel over all views: channel c, view v, pixel
 *    (x, y) at c*P + pix_off(v) + y*W_v + x, with pix_off(v) = sum of W*H of
 *    earlier views and P the total.
 *  - Per-view projection records: view v owns records rec_off(v) .. +n_v,
 *    where n_v is the size of the view's scene and rec_off(v) is the sum of
 *    earlier views' n rounded up to multiples of 64 (gs_rec_offset).
 *  - Tiles are 16x16 pixels. View v's tiles are numbered
 *    tile_base(v) + ty*gx_v + tx (gx_v = ceil(W_v/16)), after all earlier views.
 *  - Pose convention: T_cw maps world to camera, row-major [R | t]. The pose
 *    gradient is w.r.t. the twist xi = (rho, phi) of a left perturbation
 *    T <- Exp(xi) T.
 *  - Not thread-safe per context; concurrent calls on one context race.
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gs_status;
enum {
  GS_OK = 0,
  GS_E_ARG = 1,
  GS_E_CAPACITY = 2,
  GS_E_HIP = 3,
  GS_E_UNSUPPORTED = 4
};

#define GS_MAX_VIEWS 32
#define GS_TILE 16

/* Pinhole camera. 80 bytes, the same layout on host and device. */
typedef struct gs_camera {
  int32_t width, height;
  float fx, fy, cx, cy;
  float z_near; /* Gaussians with camera z <= z_near are culled */
  float pad_;
  float T_cw[12]; /* world -> camera, row-major 3x4 */
} gs_camera;

/* A batch of V views over S scenes. All Gaussians of all scenes are packed in
 * one gs_gaussians; scene s owns [scene_begin[s], scene_begin[s+1]). */
typedef struct gs_views {
  int32_t n_views;              /* 1 .. GS_MAX_VIEWS */
  int32_t n_scenes;             /* >= 1 */
  int64_t n_gaussians;          /* total Gaussians of all scenes (= gs_gaussians.n);
                                   0 is allowed in gs_project, gs_bin_sort, the
                                   render and loss calls and gs_render_bwd: their
                                   arrays sized by it (m = 0 records included)
                                   may be NULL, and the image is the background */
  const gs_camera* cams_host;   /* [host] V cameras: sizes (and values) */
  const gs_camera* cams_dev;    /* V cameras read by the kernels; poses may be
                                   updated in place between graph replays */
  const int32_t* view_scene;    /* [host] V scene ids; NULL = all scene 0 */
  const int64_t* scene_begin;   /* [host] S+1 offsets; NULL = {0, n_gaussians} */
} gs_views;

/* Gaussian parameters (planar). Quaternions (w,x,y,z) need not be unit. */
typedef struct gs_gaussians {
  int64_t n;                    /* total over all scenes */
  const float* mean;            /* [3][n] world position */
  const float* log_scale;       /* [3][n] */
  const float* quat;            /* [4][n] w, x, y, z */
  const float* opacity_logit;   /* [n] opacity = sigmoid(logit) */
  const float* color;           /* [3][n] RGB */
  const float* mp;              /* [n] motion probability in [0, 1] */
} gs_gaussians;

/* Projection output, m = gs_rec_count records. `rec`, `rect` and `depth_key`
 * are required when m > 0; the planar fields are optional (NULL skips them). */
typedef struct gs_proj {
  int64_t m;
  float* rec;        /* [m][12] compositing record: ux, uy, depth, opacity,
                        c1, c2, c3, mp, r, g, b, 0, where (c1, c2, c3) is the
                        conic (xx, xy, yy) times -log2(e) * (1/2, 1, 1/2), so
                        the Gaussian at offset d is exp2(c1 dx^2 + c2 dx dy +
                        c3 dy^2). Written by gs_project for every
                        record when key_hist is NULL; with key_hist set it is
                        written by gs_bin_sort's prefix path, for the selected
                        records only (the only ones the lists reference). */
  int16_t* rect;     /* [m][4] inclusive tile rect x0, y0, x1, y1; empty: x0 > x1.
                        The full-list binning clips it to the view's tile grid. */
  uint32_t* depth_key; /* [m] IEEE bits of camera z; 0xFFFFFFFF if culled/empty */
  float* mean2d;     /* [2][m] optional */
  float* conic;      /* [3][m] optional: inverse 2D covariance (xx, xy, yy) */
  float* depth;      /* [m] optional */
  float* opacity;    /* [m] optional */
  int32_t* radius;   /* [m] optional: opacity-aware support radius in pixels,
                        0 for culled records */
  uint32_t* key_hist;/* [V][4096] optional: gs_project adds the count of every
                        record with a key to bin (depth_key >> 20) of its view;
                        gs_bin_sort's prefix path reads it and resets it to zero.
                        Must be zero-filled before the first gs_project. */
  int32_t keys_only; /* [host, set by gs_project] 1 when it wrote the depth
                        keys only: with key_hist set, no planar output asked for
                        and the "exact_keys" knob off, gs_project runs a cheap
                        screen test instead of the full projection (the same
                        float32 depth key, near-plane and opacity culls, and a
                        tile rect from a bound on the footprint, so that it
                        never drops a Gaussian the full projection keeps);
                        depth_key and key_hist then cover the Gaussians that
                        pass it, and gs_bin_sort projects the records it
                        selects exactly (rect and compositing record), dropping
                        those the exact test culls. 0: depth_key and rect are
                        those of the full projection (set it to 0 when filling
                        rect and depth_key by other means). */
} gs_proj;

/* Per-tile lists. Entries are scene-local Gaussian ids; tile t's list is
 * gauss_id[tile_start[t] .. tile_start[t+1]), ordered by (depth bits, id). */
typedef struct gs_bins {
  int64_t capacity;       /* entries gauss_id can hold */
  uint32_t* gauss_id;     /* [capacity] */
  uint32_t* tile_start;   /* [T + 1] */
  uint32_t* sorted_ids;   /* [m] per view, record ids in (depth bits, id) order */
  int64_t* n_instances;   /* [1] total entries (also when above capacity) */
  int32_t* overflow;      /* [1] 1 when n_instances > capacity, else 0 */
  int32_t* incomplete;    /* [1] set by gs_render_fwd when a tile ran out of a
                             truncated list with unsaturated pixels (see max_rank) */
  int64_t max_rank;       /* > 0 with proj->key_hist set: bin only the records in
                             front of the first key-histogram boundary that has at
                             least max_rank records in front of it. Every tile list
                             is then an exact prefix of its full list; tiles of a
                             view whose lists leave out a visible record that run
                             out of their list with unsaturated pixels raise
                             `incomplete` (a view with at most max_rank visible
                             records keeps all of them and never does). A view
                             with more selected records than
                             gs_ctx_get_param("prefix_cap") gets empty lists and
                             raises `incomplete` at once. <= 0: full lists. */
  int32_t* truncated;     /* [1] required when max_rank > 0, owned by the library:
                             bit v is set by gs_bin_sort when view v's lists leave
                             out a visible record, and read by gs_render_fwd. */
  int32_t* sticky;        /* [2] optional (NULL skips): gs_bin_sort sets [0] to 1 when
                             the lists overflow, gs_bin_sort and gs_render_fwd set
                             [1] to 1 when `incomplete` is raised; the library
                             never clears them, so across the replays of a
                             captured loop they record whether any iteration
                             was not exact (the caller clears them) */
} gs_bins;

/* Rendered maps (planar, see layouts). */
typedef struct gs_image {
  float* color;      /* [3][P] C + T * bg */
  float* depth;      /* [P]  sum alpha T z */
  float* mp;         /* [P]  sum alpha T m (MP channel) */
  float* T;          /* [P]  final transmittance */
  uint32_t* n_last;  /* [P]  list position after the last contributing entry */
  uint32_t* tile_work; /* [2 n_tiles + 1] optional (NULL skips), zero-filled
                          before first use, then owned by the library: tile
                          scheduling state. [0, n_tiles): written by
                          gs_render_fwd, per tile the number of list entries
                          its four 64-pixel groups (pixel rows 4i..4i+3)
                          evaluated, summed. [n_tiles, 2 n_tiles]: a launch
                          order heaviest first and a marker, dealt by
                          gs_render_fwd (and gs_render_fwd_loss) from the work
                          it just wrote when "tile_order" is on, used by the
                          next gs_render_bwd and gs_render_fwd with the same
                          tile count (scheduling only: results do not depend
                          on it). */
} gs_image;

typedef struct gs_target {
  const float* color; /* [3][P] */
  const float* depth; /* [P], 0 = missing observation */
} gs_target;

typedef struct gs_loss_params {
  float lambda_pho;    /* 0.9 (Sec. V-A) */
  float lambda_depth;  /* 0.1 */
  float eps_A;         /* w = 0 where 1 - T <= eps_A (1e-6) */
  int32_t weight_mode; /* 0: w = 1 - M/(1-T) (normalised omega); 1: w = (1-T) - M */
  int32_t grad_through_weight; /* 0: w detached; 1: also emit dmp, dT */
} gs_loss_params;

typedef struct gs_pixel_grads {
  float* dcolor; /* [3][P] */
  float* ddepth; /* [P] */
  float* dmp;    /* [P] or NULL (treated as 0) */
  float* dT;     /* [P] or NULL (treated as 0) */
  const float* view_weight; /* [V] or NULL, device, read by gs_render_bwd only:
                               view v's pixel adjoints enter the backward
                               multiplied by view_weight[v] (the incoming
                               gradient of its loss); the planes are not changed */
} gs_pixel_grads;

/* Gradients w.r.t. gs_gaussians fields (same layout) and the pose twists. */
typedef struct gs_grads {
  float* mean;          /* [3][n] */
  float* log_scale;     /* [3][n] */
  float* quat;          /* [4][n] */
  float* opacity_logit; /* [n] */
  float* color;         /* [3][n] */
  float* pose;          /* [V][6] (rho, phi) */
  int32_t pose_only;    /* 1: only `pose` is written; the others may be NULL */
  int32_t accumulate;   /* 1: add to the outputs instead of overwriting */
} gs_grads;

/* ---------------------------------------------------------------- context */
typedef struct gs_ctx gs_ctx;
const char* gs_status_str(gs_status s);
/* Creates a context on `device` (must be current when calling any op). */
gs_status gs_ctx_create(int device, gs_ctx** out);
gs_status gs_ctx_destroy(gs_ctx* ctx);
const char* gs_last_error(const gs_ctx* ctx);
/* Tuning knobs: "render_batch" (64|128|256 list entries staged per LDS batch
 * in gs_render_fwd), "bwd_batch" (32|64|128, gs_render_bwd), "bin_chunk"
 * (256|512|1024|2048 records per binning workgroup), "tile_order" (0|1,
 * default 1: when the image has tile_work, the forward deals a launch order
 * heaviest first and gs_render_bwd runs its tiles in it), "bwd_copies" (1|2|4|8, default 8: accumulators of the per-record
 * 2D adjoint in the gs_render_bwd scratch, one per group of XCDs, so atomics
 * from different XCDs do not contend for one address; summed in a fixed
 * order), "wave_cull" (0|1, default 1: in gs_render_fwd and gs_render_bwd
 * each 64-pixel wave skips the entries whose alpha >= 1/255 region misses its
 * 16x4 pixel strip; the images are bit-identical either way, the gradients
 * equal up to the order of their float atomics), "exact_keys" (0|1, default 0: 1 makes gs_project run the full projection on every Gaussian also when
 * it could write the depth keys only, see gs_proj.keys_only), and
 * "timing" (0|1, see gs_ctx_kernel_times). Values outside the supported set
 * return GS_E_ARG. */
gs_status gs_ctx_set_param(gs_ctx* ctx, const char* name, int64_t value);
/* Read-only names besides the above: "lds_limit" (LDS bytes per workgroup the
 * context uses), "prefix_cap" (selected records per view the prefix binning
 * path takes), "n_cu" (compute units the tile order deals over; 0 before the
 * first gs_render_bwd on a GPU). */
gs_status gs_ctx_get_param(const gs_ctx* ctx, const char* name, int64_t* value /*[host]*/);
/* Measurement aid. With "timing" = 1 every kernel launch is bracketed by HIP
 * events on its stream (do not capture such launches in a graph). This call
 * waits for the pending events, writes one line "kernel launches total_ms" per
 * kernel into buf [host] (truncated to len bytes) and clears the record. */
gs_status gs_ctx_kernel_times(gs_ctx* ctx, char* buf, size_t len);

/* Host-side layout helpers. */
int64_t gs_rec_offset(const gs_views* views, int32_t view);
int64_t gs_rec_count(const gs_views* views);
int64_t gs_tile_count(const gs_views* views);
int64_t gs_pixel_count(const gs_views* views);

enum { GS_OP_BIN_SORT = 1, GS_OP_RENDER_BWD = 2, GS_OP_LOSS = 3, GS_OP_MP_UPDATE = 4, GS_OP_MLP_TRAIN = 5,
       GS_OP_COMPACT = 6, GS_OP_MP_REG = 7, GS_OP_EDGE_WARP = 8 };
/* Scratch bytes needed by `op` for this batch; `capacity` is the list capacity
 * of gs_bins (used by GS_OP_BIN_SORT only), for GS_OP_COMPACT and
 * GS_OP_MP_REG the number of elements n (views may then be NULL), for
 * GS_OP_EDGE_WARP the number of view pairs. For GS_OP_RENDER_BWD the size
 * grows with the context's "bwd_copies" (query it after setting the knob); the
 * scratch must be zero-filled before its first use (see gs_render_bwd). */
gs_status gs_workspace_size(gs_ctx* ctx, const gs_views* views, int32_t op, int64_t capacity, size_t* bytes);

/* ---------------------------------------------------------------- the path */

/* EWA projection (the renderer implied by Sec. IV-D, "Pixel-wise static
 * confidence"): camera mean p = R mu + t, 3D covariance from log-scale and
 * quaternion, 2D covariance J R Sigma R^T J^T + 0.3 I, conic, pixel mean,
 * sigmoid opacity, opacity-aware radius ceil(sqrt(2 ln(255 o) lambda_max)),
 * tile rect of pixels floor(u) -/+ r. Culls non-finite inputs, z <= z_near,
 * det <= 0, opacity < 1/255. */
gs_status gs_project(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, gs_proj* proj, void* stream);

/* Tile binning: per-tile lists equal to a stable ascending sort of the keys
 * (tile << 32 | depth bits) with value id, i.e. lists in (depth, id) order.
 * Sorts each view's records by depth key (LSD radix), then counts, scans and
 * scatters tile instances chunk by chunk in that order. `g` is read by the
 * prefix path only (to write proj->rec of the selected records). The path
 * follows the projection: proj->key_hist set and bins->max_rank > 0 take the
 * prefix path; the full lists (max_rank <= 0) need a gs_project run with
 * key_hist NULL, and return GS_E_ARG with key_hist set (that projection wrote
 * no compositing records, and in keys_only mode no rects). */
gs_status gs_bin_sort(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, gs_proj* proj, gs_bins* bins,
                      void* ws, size_t ws_bytes, void* stream);

/* Front-to-back compositing per 16x16 tile: alpha = min(0.99, o exp(p)),
 * entries with alpha < 1/255 skipped, stop before an entry that drops T below
 * 1e-4. Writes C + T bg, D, the MP channel M, T, n_last and, when set,
 * tile_work (per-tile work, then the backward's tile order). bg is [host]
 * RGB. */
gs_status gs_render_fwd(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                        const gs_bins* bins, const float* bg, gs_image* img, void* stream);

/* MP-weighted loss, Eq. (20)-(22) and the lambda1/lambda2 terms of Eq. (27):
 * w = 1 - M/(1-T) (0 where 1-T <= eps_A), L_v = lambda_pho sum_u w |C - C_gt|_1
 * + lambda_depth sum_u w [D_gt>0] |D - D_gt| (sums over pixels). Writes loss[V]
 * (device, deterministic) and the per-pixel adjoints (sign(0) = 0). */
gs_status gs_loss(gs_ctx* ctx, const gs_views* views, const gs_image* img, const gs_target* tgt,
                  const gs_loss_params* params /*[host]*/, float* loss, gs_pixel_grads* pg, void* ws,
                  size_t ws_bytes, void* stream);

/* gs_render_fwd followed by gs_loss in one pass: the loss and the pixel
 * adjoints are formed in the forward's epilogue from the values it writes to
 * `img`, with the targets read while the tile composites. `img` and `pg` get
 * exactly what the two calls would write; `loss` differs from gs_loss's only
 * in the order of its float64 sum (one partial per tile instead of per 256
 * pixels; still run-to-run identical). `ws` of
 * gs_workspace_size(GS_OP_LOSS). Same errors as the two calls. */
gs_status gs_render_fwd_loss(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                             const gs_bins* bins, const float* bg, gs_image* img, const gs_target* tgt,
                             const gs_loss_params* params /*[host]*/, float* loss, gs_pixel_grads* pg, void* ws,
                             size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): gs_render_fwd_loss
 * without a workspace argument, with the same results. Its per-tile float64
 * loss partials live in a static device array of 256 KiB (32768 tiles) that
 * each GPU the library runs on holds until the process ends; a batch with
 * more tiles returns GS_E_UNSUPPORTED before anything is enqueued. The
 * array's device address is resolved on the first call made with a device
 * current. The call allocates nothing (no hipMalloc, no host allocation; the
 * "timing" knob is ignored inside it). Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller. */
gs_status gs_render_fwd_loss_static(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                                    const gs_bins* bins, const float* bg, gs_image* img, const gs_target* tgt,
                                    const gs_loss_params* params /*[host]*/, float* loss, gs_pixel_grads* pg,
                                    void* stream);

/* Adjoint of render + projection for the objective sum_v L_v, to all Gaussian
 * parameters and one pose twist per view (Sec. IV-D: Gaussians and poses are
 * optimised jointly). Transmittance is recomputed back from T_final. `ws` of
 * gs_workspace_size(GS_OP_RENDER_BWD), zero-filled before first use; each
 * call leaves it zero-filled. With img->tile_work set (and "tile_order" on)
 * the tiles run in the order the forward dealt, heaviest first; the gradients
 * differ only in the order of their float atomics. When the lists overflowed
 * (the overflow flag is set) or no Gaussian is listed, every gradient and the
 * pose twists are written as zeros; with grads->accumulate set the outputs
 * are then left as they were. */
gs_status gs_render_bwd(gs_ctx* ctx, const gs_views* views, const gs_gaussians* g, const gs_proj* proj,
                        const gs_bins* bins, const gs_image* img, const gs_pixel_grads* pg, const float* bg,
                        gs_grads* grads, void* ws, size_t ws_bytes, void* stream);

/* Synchronises `stream` and reports GS_E_CAPACITY with *required = n_instances
 * when the lists overflowed; *incomplete = the gs_render_fwd flag. */
gs_status gs_bins_check(gs_ctx* ctx, const gs_bins* bins, int64_t* required /*[host]*/,
                        int32_t* incomplete /*[host], nullable*/, void* stream);

/* ---------------------------------------------------------------- MP update */
typedef struct gs_mp_frame {
  const int32_t* instance_id; /* [P] 0 = background, 1..K = instance mask id */
  int32_t n_inst;             /* K, 0 .. 15 */
  const float* inst_prior;    /* [K+1] mu(cls_k); [0] = mu(bg)   (Eq. 2) */
  const float* inst_conf;     /* [K+1] c_k; [0] = c_bg           (Eq. 2, 7) */
  int32_t seg_updated;        /* 1 if the prior was refreshed at this frame (Eq. 17) */
  const float* mlp_mp;        /* [P] nullable: per-pixel M_p from the surrogate */
} gs_mp_frame;

typedef struct gs_mp_params {
  float lambda_e;    /* Eq. (4) */
  float sigma_small; /* region mean replaces e when sigma_e < sigma_small (Eq. 5 note) */
  float e_floor;     /* lower bound of e_ub */
  float sigma_g;     /* Eq. (7) */
  float sigma_c;     /* Eq. (11) */
  float lambda_u;    /* Eq. (10) */
  float eps;         /* Eq. (10) */
  float alpha_min, alpha_max; /* Eq. (11) */
  float rho;         /* Eq. (17) */
  float radius_px;   /* association radius (Eq. 1), <= 4 */
  float sigma_w;     /* soft association kernel width */
  float beta_color;  /* photometric share of the residual cue */
  float prune_above; /* prune flag M > prune_above */
  float logodds_eps, logodds_max; /* log-odds variant */
  int32_t mode;      /* 0: exponential smoothing (Eq. 9); 1: log-odds variant */
  int32_t u_norm;    /* 0: min-max over observed Gaussians; 1: / (ln 2 + lambda_u/4) */
} gs_mp_params;

typedef struct gs_mp_out {
  float* U_tilde;    /* [n] normalised uncertainty (0 when unobserved) */
  float* alpha;      /* [n] rate alpha' used (0 when unobserved) */
  uint8_t* dynamic;  /* [n] M^t > tau (Eq. 12) */
  uint8_t* prune;    /* [n] M^t > prune_above */
  float* M_p;        /* [P] nullable: fused per-pixel MP (Eq. 6) */
  float* e;          /* [P] nullable: residual cue */
  float* stats;      /* [8]: U_bar, tau, n_obs, n_dyn, n_prune, U_min, U_max, median */
  float* judge;      /* [2] nullable: with a surrogate M_p (gs_mp_frame.mlp_mp), the
                        sum of |M_p(surrogate) - M_p(plain cue)| over the pixels
                        with observed depth, and their count (the plain cue is
                        still formed, as the surrogate's error judge; the sum
                        is accumulated with float atomics, so its last bits
                        vary); 0 and 0 without a surrogate */
} gs_mp_out;

/* One frame of the temporal MP update for a single view (views->n_views = 1).
 * Region statistics of the residual e = |D - D_gt| + beta |C - C_gt|_1 (Eq. 4),
 * MP_geo (Eq. 5), fusion with the instance prior (Eq. 2, 6, 7), per-Gaussian
 * aggregation over valid pixels within radius_px of the projected mean (Eq. 1,
 * 8), uncertainty and rate (Eq. 10, 11, 17), the state update (Eq. 9 or the
 * log-odds variant) applied in place to `mp` of the view's scene, then the
 * lower-median threshold tau = max(median, 0.5) and labels (Eq. 12) and the
 * frame uncertainty (Eq. 13). `proj` must carry mean2d. */
gs_status gs_mp_update(gs_ctx* ctx, const gs_views* views, const gs_proj* proj, const gs_image* img,
                       const gs_target* tgt, const gs_mp_frame* frame, const gs_mp_params* params /*[host]*/,
                       float* mp, gs_mp_out* out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- the further terms of the objective
 * With the photometric and depth terms of gs_loss they make the mapping
 * objective L_G = l1 L_pho + l2 L_depth + l3 L_MP + l4 L_edge (Eq. (27);
 * l3 = 500, l4 = 300 in Sec. V-A). */

/* MP-based motion consistency, Eq. (23)-(24): lambda sum_k (1 - M_k)
 * |mu_k - mu_hat_k|^2 with mu_hat_k = R mu_prev_k + t, [R | t] = T [host,
 * row-major 3x4] the relative motion that carries the previous means into the
 * current frame's coordinates (NULL: identity, for means kept in one world
 * frame). Writes lambda L_MP to loss[0] (device, deterministic) and ADDS
 * 2 lambda (1 - M_k)(mu_k - mu_hat_k) to dmean [3][n] (MP gets no gradient:
 * it is a state). mean, mean_prev [3][n], mp [n]. ws of
 * gs_workspace_size(GS_OP_MP_REG, n). */
gs_status gs_mp_regularizer(gs_ctx* ctx, int64_t n, const float* mean, const float* mean_prev, const float* mp,
                            const float* T /*[host] 12, nullable*/, float lambda, float* loss, float* dmean, void* ws,
                            size_t ws_bytes, void* stream);

/* MP-guided edge-warp term, Eq. (25)-(26), for pairs (i, j) of views of the
 * batch (i, j < n_views, i != j): over the edge pixels u of frame i (Sobel
 * slope |(S_x, S_y)| / 8 of the observed depth tgt->depth above edge_thresh,
 * every pixel of the 3x3 neighbourhood observed), the observed depth lifts u
 * into camera i, T_j T_i^-1 carries it into camera j and K_j projects it to
 * u'; frame j's rendered depth img->depth and static weight w = 1 - M/(1 - T)
 * (img->mp, img->T; 0 where 1 - T <= eps_A) are sampled bilinearly at u'
 * (skipped unless the four neighbouring pixel centres are in the image and
 * the camera-j depth exceeds z_near), and loss[k] (device) = lambda sum
 * huber_delta(w (D_j(u') - D_i(u))) for pair k. The adjoint, with w held
 * constant, is ADDED to ddepth [P] (frame j's pixels; the caller's depth
 * adjoint, so gs_render_bwd carries it to the Gaussians and frame j's pose)
 * and, through u', ADDED to dpose [V][6] (nullable) for both frames' left
 * twists. ws of gs_workspace_size(GS_OP_EDGE_WARP, n_pairs). */
typedef struct gs_edge_pair {
  int32_t i, j;
} gs_edge_pair;
typedef struct gs_edge_params {
  float lambda;      /* l4 (300 in Sec. V-A) */
  float delta;       /* Huber threshold in metres */
  float edge_thresh; /* Sobel slope threshold in metres per pixel */
  float eps_A;       /* static weight 0 where 1 - T <= eps_A */
} gs_edge_params;
gs_status gs_edge_warp(gs_ctx* ctx, const gs_views* views, const gs_image* img, const gs_target* tgt,
                       const gs_edge_pair* pairs /*[host] n_pairs*/, int32_t n_pairs,
                       const gs_edge_params* params /*[host]*/, float* loss, float* ddepth, float* dpose, void* ws,
                       size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- epipolar verification
 * Static recovery near motion boundaries, Sec. IV-C, Eq. (18)-(19). For the
 * view pair (view1, view2) of the batch, F = K2^-T [t]_x R K1^-1 with R =
 * R2 R1^T, t = t2 - R t1 from the cameras in device memory (a relative
 * translation shorter than 1e-6 has no baseline: F = 0 and every distance is
 * NaN). Match j of frame-1 pixel (p1[j], p1[m + j]) and frame-2 pixel
 * (p2[j], p2[m + j]) has the epipolar distance d[j] = |p2^T F p1| / |(a, b)|,
 * (a, b, c) = F p1 (Eq. (18)), computed in double and stored as float32
 * (NaN as the positive quiet NaN, bits 0x7FC00000). Candidate i is Gaussian
 * ids[i] (an index into the packed Gaussians of `views`) with the matches
 * seg[i] .. seg[i + 1] - 1; dbar[i] is their lower median (Eq. (19)), taken
 * over the float32 bit patterns (NaN orders above +inf; NaN when there are
 * none), and state[i] one of GS_EPI_*: RESTORED when mp[ids[i]] > tau (MP
 * suppresses it) and dbar[i] < eps (1 px in Sec. V-A), KEPT when suppressed
 * but not consistent, NOT_SUPPRESSED when mp <= tau, NO_MATCHES, or INVALID
 * (id outside [0, n_gaussians), a match range outside [0, m], or 2^31 matches
 * or more). d is written for the matches of valid candidates only; the rest
 * of d is left as it was. Every decision reads mp as it was before the call; then mp of
 * each restored candidate is set to mp_restore. p1, p2 [2][m], ids [k],
 * seg [k + 1], d [m], dbar [k], state [k] (outputs), mp [n_gaussians]
 * (in/out). No workspace. */
typedef struct gs_epi_params {
  float eps;        /* restore when dbar < eps pixels */
  float tau;        /* MP suppresses a Gaussian when mp > tau */
  float mp_restore; /* the MP a restored Gaussian gets (0: fully static) */
} gs_epi_params;
enum { GS_EPI_KEPT = 0, GS_EPI_RESTORED = 1, GS_EPI_NOT_SUPPRESSED = 2, GS_EPI_NO_MATCHES = 3, GS_EPI_INVALID = 4 };
gs_status gs_epipolar_verify(gs_ctx* ctx, const gs_views* views, int32_t view1, int32_t view2, const float* p1,
                             const float* p2, int64_t m, const int32_t* ids, const int64_t* seg, int64_t k,
                             const gs_epi_params* params /*[host]*/, float* d, float* dbar, uint8_t* state,
                             float* mp, void* stream);

/* ---------------------------------------------------------------- semantic-on-demand scheduling
 * Sec. IV-B, Eq. (13)-(17): whether to refresh the instance prior at a frame.
 * Host logic only (no device work, no stream): the inputs are the frame
 * uncertainty U_bar (Eq. (13), stats[0] of the most recent gs_mp_update) and
 * the candidates of the frame's epipolar verification (dbar and state of
 * gs_epipolar_verify, copied to the host). The verified correspondences are
 * the candidates MP labels static (state GS_EPI_NOT_SUPPRESSED) with a finite
 * median; e_bar is the mean of their medians (0 when there are none),
 * R = clip(e_bar / e_ref, 0, 1) (Eq. (14)), S = w_u U_bar + w_r R (Eq. (15)),
 * and the prior is refreshed when S > theta or dt >= n_max (Eq. (16)), dt
 * being the frames since the last refresh including this one. The caller
 * passes refresh as gs_mp_frame.seg_updated of this frame's update (Eq.
 * (17)) and reuses the last refreshed instance masks otherwise. GS_E_ARG for
 * negative weights, weights that do not sum to 1 (within 1e-6), e_ref <= 0,
 * n_max < 1. */
typedef struct gs_sched_params {
  float w_u, w_r;  /* Eq. (15); 0.5 each */
  float theta;     /* Eq. (16); 0.5 */
  float e_ref;     /* Eq. (14) in pixels; 2 */
  int32_t n_max;   /* Eq. (16); 10 */
} gs_sched_params;
typedef struct gs_sched_state {
  int32_t dt;        /* frames since the last refresh; start at n_max so the first frame refreshes */
  int32_t n_refresh; /* refreshes so far */
  float S, R, e_bar; /* the last decision's score and inputs */
} gs_sched_state;
gs_status gs_sched_decide(const gs_sched_params* params, gs_sched_state* state /*[host] in/out*/, float U_bar,
                          const float* dbar /*[host] k*/, const uint8_t* epi_state /*[host] k*/, int64_t k,
                          int32_t* refresh /*[host] out*/);

/* ---------------------------------------------------------------- measurement
 * Not part of the method: the atomic roofline of gs_render_bwd's 2D-adjoint
 * accumulation. n_ops float atomicAdds of 1.0 in groups of ten consecutive
 * floats (one record's ten adjoint components, served by ten adjacent lanes)
 * on records hash(group) % n_records of acc [copies][n_records][10] (device,
 * the caller's; each workgroup uses the copy of the XCD it runs on, as the
 * backward's "bwd_copies" do). Time it with events on `stream`. */
gs_status gs_measure_atomics(gs_ctx* ctx, float* acc, int64_t n_records, int64_t n_ops, int32_t copies,
                             void* stream);

/* ---------------------------------------------------------------- pruning
 * The mapping window prunes Gaussians whose MP after gs_mp_update exceeds a
 * threshold (the config-3 option `prune_above` flags them; not in the paper,
 * which suppresses and later recovers dynamic Gaussians, Sec. IV-C), and the
 * map is then compacted. gs_compact removes the elements with drop[i] != 0
 * from n_planes float planes of length n at once, keeping the order of the
 * rest: dst[p][j] = src[p][i_j] for the kept indices i_0 < i_1 < ... . The
 * planes are given as [host] arrays of device pointers (the Gaussian
 * parameters, the MP state, optimiser moments: any per-Gaussian float plane);
 * src and dst must not overlap. *n_out (device) gets the number kept. With
 * seg_out set, seg_begin [host] holds the n_seg + 1 offsets of contiguous
 * scenes (0 = seg_begin[0] <= ... <= seg_begin[n_seg] = n) and seg_out
 * (device) gets their new offsets (the kept elements in front of each).
 * Limits: n_planes <= GS_COMPACT_MAX_PLANES, n_seg <= GS_COMPACT_MAX_SEGS
 * (GS_E_UNSUPPORTED beyond). ws of gs_workspace_size(GS_OP_COMPACT, n). */
#define GS_COMPACT_MAX_PLANES 64
#define GS_COMPACT_MAX_SEGS 32
gs_status gs_compact(gs_ctx* ctx, const uint8_t* drop, int64_t n, int32_t n_planes,
                     const float* const* src /*[host] n_planes*/, float* const* dst /*[host] n_planes*/,
                     const int64_t* seg_begin /*[host] n_seg + 1, nullable*/, int32_t n_seg, int64_t* seg_out,
                     int64_t* n_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- learned MP surrogate
 * Not in the paper: a per-pixel MLP 8 -> 32 -> 32 -> 1 (ReLU, sigmoid) that
 * stands in for the geometric cue. Weights are used as bfloat16 copies of
 * float32 masters; biases and accumulation are float32. */
typedef struct gs_mlp {
  float* master;   /* [1377] float32: W1[32][8], b1[32], W2[32][32], b2[32], W3[32], b3[1] */
  uint16_t* w_bf16;/* [1312] bfloat16 copies of W1, W2, W3 (round to nearest even) */
  float* adam_m;   /* [1377] */
  float* adam_v;   /* [1377] */
} gs_mlp;
#define GS_MLP_PARAMS 1377
#define GS_MLP_WEIGHTS 1312

/* x[8][P] = [C - C_gt (3), (D - D_gt)[D_gt > 0] / 0.1, M, T, D / 4, MP_ins]. */
gs_status gs_mlp_features(gs_ctx* ctx, const gs_views* views, const gs_image* img, const gs_target* tgt,
                          const gs_mp_frame* frame, float* x, void* stream);
/* Refreshes w_bf16 from master (round to nearest even). */
gs_status gs_mlp_sync(gs_ctx* ctx, gs_mlp* mlp, void* stream);
/* y[P] = sigmoid(W3 relu(W2 relu(W1 x + b1) + b2) + b3). */
gs_status gs_mlp_fwd(gs_ctx* ctx, const gs_mlp* mlp, const float* x, float* y, int64_t P, void* stream);
/* One Adam step (beta 0.9/0.999, eps 1e-8) on the mean binary cross-entropy
 * against label[P]; `step` is the 1-based step count; loss[1] (device) gets
 * the loss before the step; grad[1377] (device, nullable) gets the gradient. */
gs_status gs_mlp_train_step(gs_ctx* ctx, gs_mlp* mlp, const float* x, const float* label, int64_t P,
                            float lr, int32_t step, float* loss, float* grad, void* ws, size_t ws_bytes,
                            void* stream);

/* ---------------------------------------------------------------- optimisation steps
 * The joint optimisation of Gaussian parameters and camera poses (Sec. IV-D)
 * as first-order steps on the gradients of gs_render_bwd. (The paper refines
 * poses with Levenberg-Marquardt; this library takes Adam steps on the pose
 * twist and retracts them onto SE(3).) */
typedef struct gs_adam_group {
  float* param;       /* [n] updated in place */
  const float* grad;  /* [n] */
  float* m;           /* [n] first moment, zero before the first step */
  float* v;           /* [n] second moment, zero before the first step */
  int64_t n;
  float lr;
} gs_adam_group;
typedef struct gs_adam_params {
  float beta1, beta2, eps;
  int32_t step;            /* 1-based step count of the bias correction */
  int32_t* step_dev;       /* nullable, device: when set the step count is read
                              from here at run time (a captured graph replays
                              with it advancing); `step` is ignored */
  int32_t advance;         /* with step_dev: 1 adds one to *step_dev before the
                              step (inside the Adam kernel when it is a single
                              workgroup), so a replayed graph advances its own
                              count; 0 reads it as it is */
} gs_adam_params;
#define GS_ADAM_MAX_GROUPS 8
/* Adam (Kingma and Ba 2015) on up to GS_ADAM_MAX_GROUPS device arrays in one
 * launch: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * param -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * groups [host]; GS_E_ARG for NULL arrays, n < 0, step < 1 (without step_dev)
 * or too many groups. A device step count below 1 is taken as 1. */
gs_status gs_adam_step(gs_ctx* ctx, const gs_adam_group* groups, int32_t n_groups, const gs_adam_params* params,
                       void* stream);
/* Left retraction of the pose twist on every view: T_cw[v] <- Exp(delta_v) T_cw[v]
 * with delta_v = (rho, phi) = delta[6v .. 6v + 6) (device), the SE(3)
 * exponential in closed form (Rodrigues, with series near phi = 0), the
 * rotation re-orthonormalised; delta is zeroed afterwards. `cams` is the
 * device camera table of the views (gs_views.cams_dev), updated in place. */
gs_status gs_pose_update(gs_ctx* ctx, int32_t n_views, gs_camera* cams, float* delta, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GS_H_ */
