// Internal declarations shared by the HIP sources of the WSR library.
// Everything here is gfx950-only (wave64, 160 KB LDS per CU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wsr.h"

namespace wsr {

constexpr int kWave = 64;
constexpr int kBinChunk = 2048;       // Gaussians per binning block
constexpr int kTileChunk = 14336;     // tiles per binning LDS histogram (56 KB + static < 64 KB)
constexpr int kRasterBatch = 256;     // splats staged in LDS per batch
constexpr int kItemSplats = 2048;     // a tile's list is split into raster work items of at most this many
constexpr int kProjBlock = 256;

// Camera as the kernels see it, with the per-view offsets into the
// concatenated tile, pixel and histogram spaces.
struct DevCamera {
  float R[9];
  float T[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;   // first global tile index of this view
  int32_t pad0;
  int64_t pix_base;    // first pixel of this view in the concatenated images
  int64_t hist_base;   // first entry of this view in the (block, tile) count matrix
};

// Splat record written by the projection (48 bytes, three float4):
//   r0 = (mx, my, A, B2)    centre relative to the integer origin (ox, oy), conic A, 2B
//   r1 = (C, ox, oy, amp)   conic C, integer origin as exact floats, amplitude u*w
//   r2 = (r, g, b, ext)     colour; ext packs the support half-extents (2 x fp16)
struct __align__(16) SplatRec {
  float4 r0, r1, r2;
};

// The record as stored in HBM: 64 bytes, so that no record straddles a cache
// line, with the pair-slot data the raster backward needs appended (the
// Gaussian's first Gaussian-major slot itself is in the dense goff array):
//   slot = (0, rect.x, rect.y, depth): its tile rectangle (x0 | x1 << 16,
//   y0 | y1 << 16) and its camera depth t_z as float bits (the sort key of
//   the sorted-blending baseline; positive, so the bits order like the
//   values) -- in OIT mode the opacity u instead, which Eq. 2's coverage
//   term needs beside the amplitude u w.
struct __align__(64) DevSplat {
  SplatRec s;
  uint4 slot;
};

// The caller's pair buffer (capacity entries of kPairBytes bytes): per
// (tile, Gaussian) pair a 36-byte partial 2D gradient, written by the raster
// backward at the pair's Gaussian-major slot (the Gaussian's pair offset plus
// the tile's row-major index inside the Gaussian's tile rectangle), in OIT
// mode the pair's partial dL/du through the coverage term (Gaussian-major,
// like the 2D gradient), and the per-tile lists: at each list position the
// Gaussian id and that pair's Gaussian-major slot, which the binning knows
// when it places the id, so the backward reads it with the id; then 4 bytes
// per pair for the forward's culling masks, which the backward reuses (see
// cull_mask_word in raster.hip).
constexpr int64_t kPairBytes = 52;
struct PairView {
  float3* part;        // [capacity][3] float3: (mu_x, mu_y, A) (B, C, r) (g, b, a)
  float* du;           // [capacity]
  uint2* ent;          // [capacity] list entries: (Gaussian id, Gaussian-major slot)
  uint64_t* masks;     // [capacity / 2] culling-mask words
};
__host__ __device__ inline PairView pair_view(const void* pairs, int64_t capacity) {
  char* b = static_cast<char*>(const_cast<void*>(pairs));
  PairView v;
  v.part = reinterpret_cast<float3*>(b);
  v.du = reinterpret_cast<float*>(b + 36 * capacity);
  v.ent = reinterpret_cast<uint2*>(b + 40 * capacity);  // 8-byte aligned for any capacity
  v.masks = reinterpret_cast<uint64_t*>(b + 48 * capacity);
  return v;
}

// Device-side status words (in the workspace).
struct DevFlags {
  uint32_t overflow;        // id-list capacity exceeded
  uint32_t wrapped;         // 32-bit pair count wrapped
  uint64_t total_pairs;     // pairs produced by the last binning
  uint32_t sort_overflow;   // a tile list longer than the per-tile sort takes
  uint32_t cull_masks;      // culling masks in the pair buffer: 0 none, else kCullMasks | CUT bit
};

// Value of DevFlags::cull_masks once a forward raster (without OIT) has
// stored every wave's culling masks for the current tile lists; bit 1 holds
// whether that forward used the opacity early-out.  Binning and the per-tile
// sort set it to 0.
constexpr uint32_t kCullMasks = 1u;

// Longest tile list the per-tile depth sort of the sorted-blending baseline
// holds in LDS (64-bit keys, 128 KB of the 160 KB a gfx950 workgroup may use).
constexpr int kSortMax = 16384;

struct Layout {
  int64_t n = 0;
  int32_t nv = 0;
  int32_t tile = 16;
  int32_t nblk = 1;          // binning blocks per view = ceil(n / kBinChunk)
  int32_t max_tiles_x = 1;
  int32_t max_tiles_y = 1;
  int64_t total_tiles = 0;
  int64_t total_pixels = 0;
  int64_t hist_len = 0;      // entries of the count matrix (without the trailing total)
  int64_t scan_parts = 0;
  size_t off_cams = 0, off_flags = 0, off_rec = 0, off_rect = 0, off_hist = 0, off_scan = 0,
         off_goff = 0, off_grad2d = 0, off_tstart = 0, off_tilepart = 0, off_gpart = 0, off_items = 0, off_torder = 0, off_acc = 0,
         off_oit = 0, off_acclog = 0, off_du2d = 0,
         off_queue = 0;  // work-item counters of the persistent raster launches (forward, backward)
  int64_t gpart_blocks = 0;
  size_t bytes = 0;
};

// Fill `L` (and the device cameras `dc`, host array of nv entries) from the
// arguments; returns false on invalid input.
bool make_layout(int64_t n, const wsr_camera* cams, int32_t nv, int32_t tile, Layout* L,
                 DevCamera* dc);

template <typename T>
__host__ __device__ inline T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}
template <typename T>
__host__ __device__ inline const T* at(const void* base, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(base) + off);
}

// Storage loads: fp32, fp16 or bf16 element -> float.
template <int S>
__device__ inline float load_attr(const void* p, int64_t idx);
template <>
__device__ inline float load_attr<WSR_STORE_F32>(const void* p, int64_t idx) {
  return static_cast<const float*>(p)[idx];
}
template <>
__device__ inline float load_attr<WSR_STORE_F16>(const void* p, int64_t idx) {
  return static_cast<float>(static_cast<const _Float16*>(p)[idx]);
}
template <>
__device__ inline float load_attr<WSR_STORE_BF16>(const void* p, int64_t idx) {
  const uint32_t b = static_cast<uint32_t>(static_cast<const uint16_t*>(p)[idx]) << 16;
  return __uint_as_float(b);
}

// Four consecutive storage elements (one SH coefficient, RGBA) -> float4.
template <int S>
__device__ inline float4 load_attr4(const void* p, int64_t idx4);
template <>
__device__ inline float4 load_attr4<WSR_STORE_F32>(const void* p, int64_t idx4) {
  return static_cast<const float4*>(p)[idx4];
}
template <>
__device__ inline float4 load_attr4<WSR_STORE_F16>(const void* p, int64_t idx4) {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  const h4 v = static_cast<const h4*>(p)[idx4];
  return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
}
template <>
__device__ inline float4 load_attr4<WSR_STORE_BF16>(const void* p, int64_t idx4) {
  const uint2 v = static_cast<const uint2*>(p)[idx4];
  return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                     __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
}

// Launchers (host side), one per source file.
hipError_t launch_project(const wsr_scene* sc, const wsr_params* P, const float* globals,
                          const Layout& L, void* ws, float* out_proj, hipStream_t st);
hipError_t launch_upload_cameras(const DevCamera* dc, int32_t nv, void* ws, const Layout& L,
                                 hipStream_t st);
hipError_t launch_bin(const Layout& L, void* ws, void* pairs, int64_t capacity, hipStream_t st);
hipError_t launch_raster_fwd(const Layout& L, void* ws, const void* pairs, int64_t capacity,
                             const wsr_params* P, const float* globals, float* out_rgb,
                             float* out_den, int32_t* out_count, hipStream_t st);
hipError_t launch_raster_bwd(const Layout& L, void* ws, void* pairs, int64_t capacity,
                             const wsr_params* P, const float* globals, const float* dL_drgb,
                             const float* rgb, const float* den, hipStream_t st);
hipError_t launch_project_bwd(const wsr_scene* sc, const wsr_params* P, const float* globals,
                              const Layout& L, void* ws, const void* pairs, int64_t capacity,
                              const wsr_grads* g, float* out_grad2d, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_sort_tiles(const Layout& L, void* ws, void* pairs, int64_t capacity, hipStream_t st);
hipError_t launch_raster_sorted(const Layout& L, void* ws, const void* pairs, int64_t capacity,
                                const wsr_params* P, const float* globals, float alpha_max, float alpha_min,
                                float t_min, float* out_rgb, float* out_T, hipStream_t st);
int64_t loss_workspace_bytes(const wsr_camera* cams, int32_t nv);
hipError_t launch_loss(const wsr_camera* cams, int32_t nv, const float* img, const float* target, float lambda,
                       void* ws, float* loss, float* dL, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int32_t step, float lr, float b1,
                       float b2, float eps, hipStream_t st);
// Address of the allocation-free loss's static workspace on the current
// device (WSR_LOSS_STATIC_BYTES bytes, 256-byte aligned).
hipError_t loss_static_workspace(void** out);
// Upper bound of the raster work items for an id list of `capacity` entries.
inline int64_t max_raster_items(const Layout& L, int64_t capacity) {
  return L.total_tiles + (capacity + kItemSplats - 1) / kItemSplats;
}

}  // namespace wsr
