// Step a6 of the WSR path: per-tile lists of Gaussian ids with no depth key.
// Eq. 7 is a commutative sum (Sec. 4.2), so only membership matters; this is
// the step that replaces the per-tile depth sort of 3DGS (Sec. 4.1).
//
// A counting sort by tile built from LDS histograms, with no global atomics:
//   1. bin_pass<count>: block (b, z, v) takes Gaussians [b*kBinChunk, ...) of
//      view v and counts their (tile, Gaussian) pairs into an LDS histogram
//      of the tile rows of chunk z, written contiguously as row b of the
//      block-major count matrix M[v][b][tile].
//   2. column_scan: one thread per tile turns its column of M into exclusive
//      prefixes over the blocks and produces the tile's total; a scan of the
//      totals gives every tile the start of its list (tile_start).
//   3. bin_pass<scatter>: the same blocks re-expand their pairs and place ids
//      at tile_start[t] + M[v][b][t] + an LDS-atomic cursor.
// Pairs are expanded load-balanced: per round of 256 Gaussians a block-wide
// scan of the pair counts lets every thread take every 256th pair, so one
// huge splat does not serialise on one thread.  The order of ids inside a
// tile is irrelevant to the sums (and the sums are order-insensitive up to
// float rounding).
//
// The same step also lays out the backward's per-pair scratch: every
// (view, Gaussian) gets a contiguous range of "Gaussian-major" slots, one per
// tile of its rectangle in row-major order (gauss_counts + scan), and the
// raster work items that split long tile lists (make_items + scan).
#include "wsr_internal.h"

namespace wsr {
namespace {

constexpr int kBinThreads = 256;

// Exclusive scan of one value per thread over a 256-thread block.  Returns
// the exclusive prefix; *total receives the block sum.  `sh` needs 4 words.
__device__ inline uint32_t block_scan_256(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, kWave);
    if (lane >= d) inc += o;
  }
  if (lane == kWave - 1) sh[wv] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBinThreads / kWave; ++k) {
    const uint32_t s = sh[k];
    if (k < wv) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

struct BinArgs {
  const DevCamera* cams;
  const uint2* rect;
  uint32_t* hist;              // block-major count matrix, then its column prefixes
  const uint32_t* tile_start;  // start of every tile's list (scatter pass)
  uint32_t* ids;
  int64_t n;
  int64_t capacity;
  int32_t rows_per_chunk;
};

template <bool SCATTER>
__global__ __launch_bounds__(kBinThreads) void bin_pass(BinArgs a) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t s_off[kBinThreads];
  __shared__ uint32_t s_x0[kBinThreads], s_w[kBinThreads], s_y0[kBinThreads];
  __shared__ uint32_t s_scan[4];

  const int b = blockIdx.x, z = blockIdx.y, v = blockIdx.z;
  const DevCamera& cam = a.cams[v];
  const int tiles_x = cam.tiles_x;
  const int tiles_v = cam.tiles_x * cam.tiles_y;
  const int ry0 = z * a.rows_per_chunk;
  if (ry0 >= cam.tiles_y) return;
  const int ry1 = min(ry0 + a.rows_per_chunk, cam.tiles_y);
  const int chunk_tiles = (ry1 - ry0) * tiles_x;
  const int t0 = ry0 * tiles_x;  // first tile (view-local) of the chunk
  uint32_t* row = a.hist + cam.hist_base + static_cast<int64_t>(b) * tiles_v + t0;

  for (int t = threadIdx.x; t < chunk_tiles; t += kBinThreads)
    lds[t] = SCATTER ? a.tile_start[cam.tile_base + t0 + t] + row[t] : 0u;
  __syncthreads();

  const int64_t g0 = static_cast<int64_t>(b) * kBinChunk;
  const int64_t g1 = min(g0 + kBinChunk, a.n);
  const uint2* rect = a.rect + static_cast<int64_t>(v) * a.n;
  for (int64_t base = g0; base < g1; base += kBinThreads) {
    const int64_t i = base + threadIdx.x;
    uint32_t cnt = 0, x0 = 0, w = 0, y0 = 0;
    if (i < g1) {
      const uint2 r = rect[i];
      x0 = r.x & 0xffffu;
      const uint32_t x1 = r.x >> 16;
      const int yl = max(static_cast<int>(r.y & 0xffffu), ry0);
      const int yh = min(static_cast<int>(r.y >> 16), ry1);
      w = x1 > x0 ? x1 - x0 : 0u;
      if (yh > yl && w > 0) {
        cnt = w * static_cast<uint32_t>(yh - yl);
        y0 = static_cast<uint32_t>(yl);
      }
    }
    uint32_t total;
    const uint32_t off = block_scan_256(cnt, s_scan, &total);
    s_off[threadIdx.x] = off;
    s_x0[threadIdx.x] = x0;
    s_w[threadIdx.x] = w;
    s_y0[threadIdx.x] = y0;
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < total; p += kBinThreads) {
      // largest g with s_off[g] <= p (it has a non-zero count)
      int lo = 0, hi = kBinThreads - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= p) lo = mid; else hi = mid - 1;
      }
      const uint32_t local = p - s_off[lo];
      const uint32_t ww = s_w[lo];
      const uint32_t ty = s_y0[lo] + local / ww;
      const uint32_t tx = s_x0[lo] + local % ww;
      const uint32_t t = (ty - ry0) * tiles_x + tx;
      if (!SCATTER) {
        atomicAdd(&lds[t], 1u);
      } else {
        const uint32_t pos = atomicAdd(&lds[t], 1u);
        if (pos < a.capacity) a.ids[pos] = static_cast<uint32_t>(base + lo);
      }
    }
    __syncthreads();
  }
  if (!SCATTER) {
    for (int t = threadIdx.x; t < chunk_tiles; t += kBinThreads) row[t] = lds[t];
  }
}

// One thread per tile: exclusive prefix of the tile's column of counts over
// the blocks (in place), and the tile's total into tile_start[t].
__global__ __launch_bounds__(256) void column_scan(const DevCamera* cams, int32_t nv, int32_t nblk,
                                                   int64_t total_tiles, uint32_t* hist, uint32_t* tile_start) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t > total_tiles) return;
  if (t == total_tiles) {
    tile_start[t] = 0u;
    return;
  }
  int v = 0;
  while (v + 1 < nv && cams[v + 1].tile_base <= t) ++v;
  const DevCamera& cam = cams[v];
  const int64_t tiles_v = static_cast<int64_t>(cam.tiles_x) * cam.tiles_y;
  uint32_t* col = hist + cam.hist_base + (t - cam.tile_base);
  uint32_t run = 0;
  int b = 0;
  for (; b + 8 <= nblk; b += 8) {  // eight independent loads in flight
    uint32_t c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = col[(b + k) * tiles_v];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      col[(b + k) * tiles_v] = run;
      run += c[k];
    }
  }
  for (; b < nblk; ++b) {
    const uint32_t c = col[b * tiles_v];
    col[b * tiles_v] = run;
    run += c;
  }
  tile_start[t] = run;
}

// ---- device-wide exclusive scan of uint32 (in place), 3 phases ----

__global__ __launch_bounds__(256) void scan_reduce(const uint32_t* x, int64_t len, uint32_t* parts) {
  __shared__ uint32_t sh[4];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanItems + threadIdx.x * 16;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (base + k < len) s += x[base + k];
  uint32_t total;
  block_scan_256(s, sh, &total);
  if (threadIdx.x == 0) parts[blockIdx.x] = total;
}

// Scans the per-block partial sums; with `flags`, also records the grand
// total and whether it exceeds `capacity` or 32 bits.
__global__ __launch_bounds__(1024) void scan_parts(uint32_t* parts, int64_t nparts, DevFlags* flags,
                                                   int64_t capacity) {
  __shared__ uint32_t sh[16];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  uint64_t carry = 0;
  for (int64_t c0 = 0; c0 < nparts; c0 += 1024) {
    const int64_t j = c0 + threadIdx.x;
    const uint32_t v = j < nparts ? parts[j] : 0u;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t o = __shfl_up(inc, d, kWave);
      if (lane >= d) inc += o;
    }
    if (lane == kWave - 1) sh[wv] = inc;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < wv) before += sh[k];
      tot += sh[k];
    }
    if (j < nparts) parts[j] = static_cast<uint32_t>(carry + before + inc - v);
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && flags) {
    flags->total_pairs = carry;
    flags->wrapped = carry > 0xffffffffull ? 1u : 0u;
    flags->overflow = (carry > static_cast<uint64_t>(capacity) || carry > 0xffffffffull) ? 1u : 0u;
    flags->sort_overflow = 0u;
  }
}

__global__ __launch_bounds__(256) void scan_apply(uint32_t* x, int64_t len, const uint32_t* parts) {
  __shared__ uint32_t sh[4];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanItems + threadIdx.x * 16;
  uint32_t vals[16];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    vals[k] = base + k < len ? x[base + k] : 0u;
    s += vals[k];
  }
  uint32_t total;
  uint32_t run = block_scan_256(s, sh, &total) + parts[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (base + k < len) x[base + k] = run;
    run += vals[k];
  }
}

hipError_t scan_in_place(uint32_t* x, int64_t len, uint32_t* parts, DevFlags* flags, int64_t capacity,
                         hipStream_t st) {
  const unsigned np = static_cast<unsigned>((len + kScanItems - 1) / kScanItems);
  scan_reduce<<<np, 256, 0, st>>>(x, len, parts);
  scan_parts<<<1, 1024, 0, st>>>(parts, np, flags, capacity);
  scan_apply<<<np, 256, 0, st>>>(x, len, parts);
  return hipGetLastError();
}

// Number of (tile, Gaussian) pairs of every (view, Gaussian) slot, the
// input of the scan that gives each Gaussian a contiguous range of
// Gaussian-major pair slots (the raster backward writes a partial gradient
// per pair there; the projection backward sums the range).
__global__ __launch_bounds__(256) void gauss_counts(const uint2* rect, int64_t slots, uint32_t* goff) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k > slots) return;
  if (k == slots) {
    goff[k] = 0u;
    return;
  }
  const uint2 r = rect[k];
  const uint32_t x0 = r.x & 0xffffu, x1 = r.x >> 16, y0 = r.y & 0xffffu, y1 = r.y >> 16;
  goff[k] = (x1 > x0 && y1 > y0) ? (x1 - x0) * (y1 - y0) : 0u;
}

// Copies every (view, Gaussian)'s first pair slot into its record (the
// projection stored the tile rectangle there), where the raster backward
// reads it with the rest of the record: one cache line per pair instead of
// three.
__global__ __launch_bounds__(256) void record_slots(const uint32_t* goff, int64_t slots, DevSplat* rec) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k >= slots) return;
  rec[k].slot.x = goff[k];
}

// Raster work items: tile t's list is cut into max(1, ceil(L / kItemSplats))
// items, so no single workgroup carries a tile many times heavier than the
// mean.  items[t] receives the count here and its exclusive prefix after the
// scan; items[total_tiles] ends up holding the number of items.
__global__ __launch_bounds__(256) void make_items(const uint32_t* tile_start, int64_t capacity, int64_t total_tiles,
                                                  uint32_t* items) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t > total_tiles) return;
  if (t == total_tiles) {
    items[t] = 0u;
    return;
  }
  const uint64_t cap = static_cast<uint64_t>(capacity);
  uint64_t s = tile_start[t], e = tile_start[t + 1];
  s = s < cap ? s : cap;
  e = e < cap ? e : cap;
  const uint64_t len = e > s ? e - s : 0;
  items[t] = static_cast<uint32_t>(len == 0 ? 1 : (len + kItemSplats - 1) / kItemSplats);
}

}  // namespace

hipError_t launch_bin(const Layout& L, void* ws, void* pairs, int64_t capacity, bool oit, hipStream_t st) {
  DevFlags* flags = at<DevFlags>(ws, L.off_flags);
  uint32_t* hist = at<uint32_t>(ws, L.off_hist);
  uint32_t* parts = at<uint32_t>(ws, L.off_scan);
  uint32_t* goff = at<uint32_t>(ws, L.off_goff);
  uint32_t* tstart = at<uint32_t>(ws, L.off_tstart);
  uint32_t* items = at<uint32_t>(ws, L.off_items);
  const PairView pv = pair_view(pairs, capacity);

  BinArgs a;
  a.cams = at<DevCamera>(ws, L.off_cams);
  a.rect = at<uint2>(ws, L.off_rect);
  a.hist = hist;
  a.tile_start = tstart;
  a.ids = pv.ids;
  a.n = L.n;
  a.capacity = capacity;
  // whole tile rows per LDS chunk, at most kTileChunk tiles
  a.rows_per_chunk = kTileChunk / L.max_tiles_x;
  if (a.rows_per_chunk < 1) return hipErrorInvalidValue;
  const int nchunks = (L.max_tiles_y + a.rows_per_chunk - 1) / a.rows_per_chunk;
  const size_t lds = static_cast<size_t>(a.rows_per_chunk) * L.max_tiles_x * sizeof(uint32_t);
  const dim3 grid(static_cast<unsigned>(L.nblk), static_cast<unsigned>(nchunks), static_cast<unsigned>(L.nv));

  // split-tile accumulators of the forward raster start at zero
  hipError_t e = launch_fill_zero(at<float>(ws, L.off_acc), sizeof(float) * 4 * L.total_pixels, st);
  if (e != hipSuccess) return e;
  if (oit && (e = launch_fill_zero(at<float>(ws, L.off_acclog), sizeof(float) * L.total_pixels, st)) != hipSuccess)
    return e;
  bin_pass<false><<<grid, kBinThreads, lds, st>>>(a);
  const int64_t tl = L.total_tiles + 1;
  column_scan<<<static_cast<unsigned>((tl + 255) / 256), 256, 0, st>>>(a.cams, L.nv, L.nblk, L.total_tiles, hist,
                                                                      tstart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_in_place(tstart, tl, parts, flags, capacity, st)) != hipSuccess) return e;
  bin_pass<true><<<grid, kBinThreads, lds, st>>>(a);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  // Gaussian-major pair offsets (exclusive scan of the rectangle sizes)
  const int64_t glen = L.n * L.nv + 1;
  gauss_counts<<<static_cast<unsigned>((glen + 255) / 256), 256, 0, st>>>(a.rect, L.n * L.nv, goff);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_in_place(goff, glen, parts, nullptr, 0, st)) != hipSuccess) return e;
  if (L.n * L.nv > 0) {
    record_slots<<<static_cast<unsigned>((L.n * L.nv + 255) / 256), 256, 0, st>>>(goff, L.n * L.nv,
                                                                                  at<DevSplat>(ws, L.off_rec));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }

  // raster work items per tile, then their exclusive prefix
  make_items<<<static_cast<unsigned>((tl + 255) / 256), 256, 0, st>>>(tstart, capacity, L.total_tiles, items);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return scan_in_place(items, tl, parts, nullptr, 0, st);
}

}  // namespace wsr
