// C-ABI entry points of the WSR library (declared in include/wsr.h): argument
// checks, workspace layout, and the launch sequence of each step.
#include <cmath>
#include <cstring>

#include "adam.h"
#include "wsr_internal.h"

namespace wsr {

int64_t project_bwd_blocks(int64_t n);

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

bool valid_tile(int32_t t) { return t == 8 || t == 16 || t == 32; }

int32_t to_status(hipError_t e) { return e == hipSuccess ? WSR_OK : WSR_ERR_HIP; }

}  // namespace

bool make_layout(int64_t n, const wsr_camera* cams, int32_t nv, int32_t tile, Layout* L, DevCamera* dc) {
  if (n < 0 || n > 0xffffffffLL || !cams || nv < 1 || nv > WSR_MAX_VIEWS || !valid_tile(tile)) return false;
  *L = Layout();
  L->n = n;
  L->nv = nv;
  L->tile = tile;
  L->nblk = static_cast<int32_t>(n > 0 ? (n + kBinChunk - 1) / kBinChunk : 1);
  int64_t tiles = 0, pixels = 0, hist = 0;
  for (int v = 0; v < nv; ++v) {
    const wsr_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 32767 || c.height > 32767) return false;
    if (!(c.fx > 0.f) || !(c.fy > 0.f)) return false;
    const int tx = (c.width + tile - 1) / tile, ty = (c.height + tile - 1) / tile;
    if (tx > L->max_tiles_x) L->max_tiles_x = tx;
    if (ty > L->max_tiles_y) L->max_tiles_y = ty;
    if (dc) {
      DevCamera& d = dc[v];
      std::memset(&d, 0, sizeof(d));
      for (int k = 0; k < 3; ++k) {
        for (int j = 0; j < 3; ++j) d.R[3 * k + j] = c.viewmat[4 * k + j];
        d.T[k] = c.viewmat[4 * k + 3];
      }
      d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
      d.width = c.width; d.height = c.height;
      d.tiles_x = tx; d.tiles_y = ty;
      d.tile_base = static_cast<int32_t>(tiles);
      d.pix_base = pixels;
      d.hist_base = hist;
    }
    tiles += static_cast<int64_t>(tx) * ty;
    pixels += static_cast<int64_t>(c.width) * c.height;
    hist += static_cast<int64_t>(tx) * ty * L->nblk;
  }
  if (tiles > 0x7fffffffLL) return false;
  L->total_tiles = tiles;
  L->total_pixels = pixels;
  L->hist_len = hist;
  L->scan_parts = static_cast<int64_t>(nv) * L->nblk;  // one rectangle sum per (view, binning block)
  L->gpart_blocks = project_bwd_blocks(n);
  const int64_t slots = n * nv;
  size_t off = 0;
  L->off_cams = off;     off = align256(off + sizeof(DevCamera) * WSR_MAX_VIEWS);
  L->off_flags = off;    off = align256(off + sizeof(DevFlags));
  L->off_queue = off;    off = align256(off + sizeof(uint32_t) * 2);
  L->off_rec = off;      off = align256(off + sizeof(DevSplat) * slots);
  L->off_rect = off;     off = align256(off + sizeof(uint2) * slots);
  L->off_hist = off;     off = align256(off + sizeof(uint32_t) * (hist + 1));
  L->off_scan = off;     off = align256(off + sizeof(uint32_t) * L->scan_parts);
  L->off_goff = off;     off = align256(off + sizeof(uint32_t) * (slots + 1));
  L->off_grad2d = off;   off = align256(off + sizeof(float) * 9 * slots);
  L->off_tstart = off;   off = align256(off + sizeof(uint32_t) * (tiles + 1));
  L->off_tilepart = off; off = align256(off + sizeof(float) * 4 * tiles);
  L->off_gpart = off;    off = align256(off + sizeof(double) * 2 * L->gpart_blocks);
  L->off_items = off;    off = align256(off + sizeof(uint32_t) * (tiles + 1));
  L->off_torder = off;   off = align256(off + sizeof(uint32_t) * (tiles > 0 ? tiles : 1));
  L->off_acc = off;      off = align256(off + sizeof(float) * 4 * pixels);
  L->off_oit = off;      off = align256(off + sizeof(float) * 4 * pixels);
  L->off_acclog = off;   off = align256(off + sizeof(float) * pixels);
  L->off_du2d = off;     off = align256(off + sizeof(float) * (slots > 0 ? slots : 1));
  L->bytes = off;
  return true;
}

}  // namespace wsr

using namespace wsr;

namespace {

bool scene_ok(const wsr_scene* s, int32_t weight_kind) {
  if (!s || s->n < 0 || s->sh_degree < 0 || s->sh_degree > 3) return false;
  if (s->storage < WSR_STORE_F32 || s->storage > WSR_STORE_BF16) return false;
  if (s->opacity_mode != WSR_OPACITY_LOGIT && s->opacity_mode != WSR_OPACITY_SH) return false;
  if (s->n == 0) return true;
  if (!s->means || !s->log_scales || !s->quats || !s->sh) return false;
  if (s->opacity_mode == WSR_OPACITY_LOGIT && !s->opacity_logit) return false;
  if (weight_kind == WSR_WEIGHT_LC && !s->lc_v) return false;
  return true;
}

// Raster batch sizes each tile size is built for (0 picks the default).
bool batch_ok(int32_t tile, int32_t batch) {
  if (batch == 0) return true;
  if (tile == 8) return batch == 64;
  if (tile == 16) return batch == 64 || batch == 128 || batch == 256;
  return batch == 128 || batch == 256;
}

bool params_ok(const wsr_params* p) {
  return p && p->weight_kind >= WSR_WEIGHT_DIR && p->weight_kind <= WSR_WEIGHT_LC &&
         (p->tile == 8 || p->tile == 16 || p->tile == 32) && std::isfinite(p->tau) && p->tau >= 0.f &&
         std::isfinite(p->dilation) && std::isfinite(p->near_z) && std::isfinite(p->alpha_cut) &&
         p->alpha_cut >= 0.f &&
         (p->flags & ~(WSR_FLAG_UNNORMALISED | WSR_FLAG_OIT | WSR_FLAG_PERSISTENT)) == 0 &&
         (!(p->flags & WSR_FLAG_OIT) || ((p->flags & WSR_FLAG_UNNORMALISED) == 0 && p->alpha_cut == 0.f)) &&
         batch_ok(p->tile, p->batch);
}

}  // namespace

extern "C" {

int32_t wsr_abi_version(void) { return WSR_ABI_VERSION; }

const char* wsr_status_string(int32_t status) {
  switch (status) {
    case WSR_OK: return "ok";
    case WSR_ERR_INVALID: return "invalid argument";
    case WSR_ERR_WORKSPACE: return "workspace too small";
    case WSR_ERR_CAPACITY: return "per-tile id list overflow";
    case WSR_ERR_HIP: return "HIP runtime error";
    case WSR_ERR_TILE_LIST: return "tile list longer than the per-tile sort takes";
    case WSR_ERR_STATIC: return "request larger than the static workspace of an allocation-free entry point";
    default: return "unknown status";
  }
}

int64_t wsr_workspace_bytes(int64_t n, const wsr_camera* cams, int32_t n_views, int32_t tile) {
  Layout L;
  if (!make_layout(n, cams, n_views, tile, &L, nullptr)) return -1;
  return static_cast<int64_t>(L.bytes);
}

int32_t wsr_project(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views, const wsr_params* params,
                    const float* globals, void* ws, int64_t ws_bytes, float* out_proj, void* stream) {
  if (!params_ok(params) || !scene_ok(scene, params->weight_kind) || !globals || !ws) return WSR_ERR_INVALID;
  Layout L;
  DevCamera dc[WSR_MAX_VIEWS];
  if (!make_layout(scene->n, cams, n_views, params->tile, &L, dc)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = launch_upload_cameras(dc, n_views, ws, L, st);
  if (e == hipSuccess) e = launch_project(scene, params, globals, L, ws, out_proj, st);
  return to_status(e);
}

int64_t wsr_pair_bytes(void) { return kPairBytes; }

static bool pairs_ok(const void* pairs, int64_t capacity) {
  return capacity >= 0 && capacity <= 0xffffffffLL &&
         (capacity == 0 || (pairs && (reinterpret_cast<uintptr_t>(pairs) & 255u) == 0));
}

int32_t wsr_bin(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n, void* ws,
                int64_t ws_bytes, void* pairs, int64_t capacity, void* stream) {
  if (!params_ok(params) || !ws || !pairs_ok(pairs, capacity)) return WSR_ERR_INVALID;
  Layout L;
  if (!make_layout(n, cams, n_views, params->tile, &L, nullptr)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  return to_status(launch_bin(L, ws, pairs, capacity, static_cast<hipStream_t>(stream)));
}

int32_t wsr_render_fwd(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                       const float* globals, void* ws, int64_t ws_bytes, void* pairs,
                       int64_t capacity, float* out_rgb, float* out_den, int32_t* out_count, void* stream) {
  if (!params_ok(params) || !globals || !ws || !out_rgb || !out_den || !pairs_ok(pairs, capacity))
    return WSR_ERR_INVALID;
  Layout L;
  if (!make_layout(n, cams, n_views, params->tile, &L, nullptr)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  return to_status(launch_raster_fwd(L, ws, pairs, capacity, params, globals, out_rgb, out_den, out_count,
                                     static_cast<hipStream_t>(stream)));
}

int32_t wsr_raster_bwd(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                       const float* globals, void* ws, int64_t ws_bytes, void* pairs, int64_t capacity,
                       const float* dL_drgb, const float* rgb, const float* den, void* stream) {
  if (!params_ok(params) || !globals || !ws || !dL_drgb || !rgb || !den || !pairs_ok(pairs, capacity))
    return WSR_ERR_INVALID;
  Layout L;
  if (!make_layout(n, cams, n_views, params->tile, &L, nullptr)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  return to_status(launch_raster_bwd(L, ws, pairs, capacity, params, globals, dL_drgb, rgb, den,
                                     static_cast<hipStream_t>(stream)));
}

int32_t wsr_project_bwd(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views, const wsr_params* params,
                        const float* globals, void* ws, int64_t ws_bytes, const void* pairs, int64_t capacity,
                        const wsr_grads* grads, float* out_grad2d, void* stream) {
  if (!params_ok(params) || !scene_ok(scene, params->weight_kind) || !globals || !ws || !grads || !grads->globals ||
      !pairs_ok(pairs, capacity))
    return WSR_ERR_INVALID;
  if (scene->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->sh)) return WSR_ERR_INVALID;
  Layout L;
  if (!make_layout(scene->n, cams, n_views, params->tile, &L, nullptr)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  return to_status(launch_project_bwd(scene, params, globals, L, ws, pairs, capacity, grads, out_grad2d,
                                      static_cast<hipStream_t>(stream)));
}

int32_t wsr_project_bwd_adam(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views,
                             const wsr_params* params, const float* globals, void* ws, int64_t ws_bytes,
                             const void* pairs, int64_t capacity, const wsr_grads* m, const wsr_grads* v,
                             const wsr_adam_params* adam, float* grad_globals, float* out_grad2d,
                             void* stream) {
  if (!params_ok(params) || !scene_ok(scene, params->weight_kind) || !globals || !ws || !m || !v || !adam ||
      !grad_globals || !pairs_ok(pairs, capacity))
    return WSR_ERR_INVALID;
  if (scene->storage != WSR_STORE_F32 || adam->step < 1 || !(adam->beta1 >= 0.f && adam->beta1 < 1.f) ||
      !(adam->beta2 >= 0.f && adam->beta2 < 1.f))
    return WSR_ERR_INVALID;
  if (scene->n > 0 && (!m->means || !m->log_scales || !m->quats || !m->sh || !v->means || !v->log_scales ||
                       !v->quats || !v->sh))
    return WSR_ERR_INVALID;
  Layout L;
  if (!make_layout(scene->n, cams, n_views, params->tile, &L, nullptr)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  FusedAdam f;
  f.m = *m;
  f.v = *v;
  const float lr[7] = {adam->lr_means, adam->lr_log_scales, adam->lr_quats, adam->lr_sh0, adam->lr_shN,
                       adam->lr_opacity_logit, adam->lr_lc_v};
  for (int k = 0; k < 7; ++k) f.lr[k] = lr[k];
  f.step = make_adam_step(adam->step, adam->beta1, adam->beta2, adam->eps);
  return to_status(launch_project_bwd_adam(scene, params, globals, L, ws, pairs, capacity, f, grad_globals,
                                           out_grad2d, static_cast<hipStream_t>(stream)));
}

int32_t wsr_render_bwd(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views, const wsr_params* params,
                       const float* globals, void* ws, int64_t ws_bytes, void* pairs, int64_t capacity,
                       const float* dL_drgb, const float* rgb, const float* den, const wsr_grads* grads,
                       float* out_grad2d, void* stream) {
  if (!params_ok(params) || !scene_ok(scene, params->weight_kind) || !grads || !grads->globals)
    return WSR_ERR_INVALID;
  if (scene->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->sh)) return WSR_ERR_INVALID;
  const int32_t s = wsr_raster_bwd(cams, n_views, params, scene->n, globals, ws, ws_bytes, pairs, capacity,
                                   dL_drgb, rgb, den, stream);
  if (s != WSR_OK) return s;
  return wsr_project_bwd(scene, cams, n_views, params, globals, ws, ws_bytes, pairs, capacity, grads, out_grad2d,
                         stream);
}

int32_t wsr_pair_count(const void* ws, int64_t ws_bytes, int64_t* out_total, void* stream) {
  if (!ws || !out_total || ws_bytes < static_cast<int64_t>(sizeof(DevCamera) * WSR_MAX_VIEWS + sizeof(DevFlags)))
    return WSR_ERR_INVALID;
  Layout L;  // flags sit at a fixed offset after the camera table
  wsr_camera probe = {};
  probe.width = probe.height = 1;
  probe.fx = probe.fy = 1.f;
  make_layout(0, &probe, 1, 16, &L, nullptr);
  DevFlags f;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&f, at<DevFlags>(ws, L.off_flags), sizeof(f), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return WSR_ERR_HIP;
  *out_total = static_cast<int64_t>(f.total_pairs);
  return WSR_OK;
}

int32_t wsr_check(const void* ws, int64_t ws_bytes, void* stream) {
  if (!ws || ws_bytes < static_cast<int64_t>(sizeof(DevCamera) * WSR_MAX_VIEWS + sizeof(DevFlags)))
    return WSR_ERR_INVALID;
  Layout L;
  wsr_camera probe = {};
  probe.width = probe.height = 1;
  probe.fx = probe.fy = 1.f;
  make_layout(0, &probe, 1, 16, &L, nullptr);
  DevFlags f;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&f, at<DevFlags>(ws, L.off_flags), sizeof(f), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return WSR_ERR_HIP;
  if (f.overflow) return WSR_ERR_CAPACITY;
  return f.sort_overflow ? WSR_ERR_TILE_LIST : WSR_OK;
}

int32_t wsr_sort_tiles(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                       void* ws, int64_t ws_bytes, void* pairs, int64_t capacity, void* stream) {
  static_assert(kSortMax == WSR_SORT_MAX, "sort limit");
  if (!params_ok(params) || params->alpha_cut != 0.f || (params->flags & WSR_FLAG_OIT) || !ws ||
      !pairs_ok(pairs, capacity))
    return WSR_ERR_INVALID;
  Layout L;
  if (!make_layout(n, cams, n_views, params->tile, &L, nullptr)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  const hipError_t e = launch_sort_tiles(L, ws, pairs, capacity, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? WSR_OK : WSR_ERR_HIP;
}

int32_t wsr_render_sorted(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                          const float* globals, const wsr_blend* blend, void* ws, int64_t ws_bytes,
                          const void* pairs, int64_t capacity, float* out_rgb, float* out_T, void* stream) {
  if (!params_ok(params) || params->weight_kind != WSR_WEIGHT_DIR || params->alpha_cut != 0.f ||
      (params->flags & WSR_FLAG_OIT) || !globals ||
      !blend || !ws || !out_rgb ||
      !out_T || !pairs_ok(pairs, capacity))
    return WSR_ERR_INVALID;
  if (!(blend->alpha_max > 0.f && blend->alpha_max <= 1.f) || !(blend->alpha_min >= 0.f) ||
      !(blend->t_min >= 0.f))
    return WSR_ERR_INVALID;
  Layout L;
  if (!make_layout(n, cams, n_views, params->tile, &L, nullptr)) return WSR_ERR_INVALID;
  if (ws_bytes < static_cast<int64_t>(L.bytes)) return WSR_ERR_WORKSPACE;
  const hipError_t e = launch_raster_sorted(L, ws, pairs, capacity, params, globals, blend->alpha_max,
                                            blend->alpha_min, blend->t_min, out_rgb, out_T,
                                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? WSR_OK : WSR_ERR_HIP;
}

static bool loss_cams_ok(const wsr_camera* cams, int32_t n_views) {
  if (!cams || n_views < 1 || n_views > WSR_MAX_VIEWS) return false;
  for (int v = 0; v < n_views; ++v)
    if (cams[v].width < 1 || cams[v].height < 1 || cams[v].width > 32767 || cams[v].height > 32767) return false;
  return true;
}

int64_t wsr_loss_workspace_bytes(const wsr_camera* cams, int32_t n_views) {
  if (!loss_cams_ok(cams, n_views)) return -1;
  return loss_workspace_bytes(cams, n_views);
}

int32_t wsr_loss(const wsr_camera* cams, int32_t n_views, const float* img, const float* target, float lambda,
                 void* ws, int64_t ws_bytes, float* loss, float* dL_dimg, void* stream) {
  if (!loss_cams_ok(cams, n_views) || !img || !target || !ws || !loss || !dL_dimg) return WSR_ERR_INVALID;
  if (!(lambda >= 0.f && lambda <= 1.f)) return WSR_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return WSR_ERR_INVALID;
  if (ws_bytes < loss_workspace_bytes(cams, n_views)) return WSR_ERR_WORKSPACE;
  const hipError_t e = launch_loss(cams, n_views, img, target, lambda, ws, loss, dL_dimg,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? WSR_OK : WSR_ERR_HIP;
}

int32_t wsr_loss_noalloc(const wsr_camera* cams, int32_t n_views, const float* img, const float* target,
                         float lambda, float* loss, float* dL_dimg, void* stream) {
  if (!loss_cams_ok(cams, n_views) || !img || !target || !loss || !dL_dimg) return WSR_ERR_INVALID;
  if (!(lambda >= 0.f && lambda <= 1.f)) return WSR_ERR_INVALID;
  if (loss_workspace_bytes(cams, n_views) > static_cast<int64_t>(WSR_LOSS_STATIC_BYTES)) return WSR_ERR_STATIC;
  void* ws = nullptr;
  if (loss_static_workspace(&ws) != hipSuccess) return WSR_ERR_HIP;
  const hipError_t e = launch_loss(cams, n_views, img, target, lambda, ws, loss, dL_dimg,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? WSR_OK : WSR_ERR_HIP;
}

int32_t wsr_adam(float* param, const float* grad, float* m, float* v, int64_t n, int32_t step, float lr,
                 float beta1, float beta2, float eps, void* stream) {
  if (n < 0 || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f)) return WSR_ERR_INVALID;
  if (n > 0 && (!param || !grad || !m || !v)) return WSR_ERR_INVALID;
  const hipError_t e = launch_adam(param, grad, m, v, n, step, lr, beta1, beta2, eps,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? WSR_OK : WSR_ERR_HIP;
}

}  // extern "C"
