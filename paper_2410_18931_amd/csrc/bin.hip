// Step a6 of the WSR path: per-tile lists of Gaussian ids with no depth key.
// Eq. 7 is a commutative sum (Sec. 4.2), so only membership matters; this is
// the step that replaces the per-tile depth sort of 3DGS (Sec. 4.1).
//
// A counting sort by tile, built from LDS histograms instead of global
// atomics:
//   1. bin_count: block (b, z, v) takes Gaussians [b*kBinChunk, ...) of view v
//      and counts their (tile, Gaussian) pairs into an LDS histogram of the
//      tile rows of chunk z.  The histogram is stored as column b of a
//      tile-major count matrix M[v][tile][b].
//   2. an exclusive scan over M (tile-major) gives every (tile, block) segment
//      its start; tile t of view v spans [M[v][t][0], M[v][t+1][0]).
//   3. bin_scatter: the same blocks re-expand their pairs and place ids at
//      start + LDS-atomic cursor.
// Pairs are expanded load-balanced: per round of 256 Gaussians a block-wide
// scan of the pair counts lets every thread take every 256th pair, so one
// huge splat does not serialise on one thread.
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
  uint32_t* hist;
  const uint32_t* goff;   // Gaussian-major pair offsets per (view, Gaussian)
  uint32_t* ids;
  uint32_t* slot;
  int64_t n;
  int64_t capacity;
  int32_t nblk;
  int32_t rows_per_chunk;
};

// Shared expansion loop.  SCATTER = false counts, true places ids.
template <bool SCATTER>
__global__ __launch_bounds__(kBinThreads) void bin_pass(BinArgs a) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t s_off[kBinThreads + 1];
  __shared__ uint32_t s_x0[kBinThreads], s_w[kBinThreads], s_y0[kBinThreads], s_goff[kBinThreads];
  __shared__ uint32_t s_scan[4];

  const int b = blockIdx.x, z = blockIdx.y, v = blockIdx.z;
  const DevCamera& cam = a.cams[v];
  const int tiles_x = cam.tiles_x;
  const int ry0 = z * a.rows_per_chunk;
  if (ry0 >= cam.tiles_y) return;
  const int ry1 = min(ry0 + a.rows_per_chunk, cam.tiles_y);
  const int chunk_tiles = (ry1 - ry0) * tiles_x;
  uint32_t* col = a.hist + cam.hist_base + static_cast<int64_t>(ry0) * tiles_x * a.nblk + b;

  for (int t = threadIdx.x; t < chunk_tiles; t += kBinThreads)
    lds[t] = SCATTER ? col[static_cast<int64_t>(t) * a.nblk] : 0u;
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
    // first Gaussian-major slot of this Gaussian's pairs in this chunk: its
    // pairs are enumerated row by row over its rectangle, so the rows of the
    // chunk start after (yl - y0_rect) * w of them
    if (SCATTER && i < g1) {
      const uint2 r = rect[i];
      const uint32_t yr = r.y & 0xffffu;
      s_goff[threadIdx.x] = a.goff[static_cast<int64_t>(v) * a.n + i] + (y0 > yr ? (y0 - yr) * w : 0u);
    }
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
        if (pos < a.capacity) {
          a.ids[pos] = static_cast<uint32_t>(base + lo);
          a.slot[pos] = s_goff[lo] + local;
        }
      }
    }
    __syncthreads();
  }
  if (!SCATTER) {
    for (int t = threadIdx.x; t < chunk_tiles; t += kBinThreads)
      col[static_cast<int64_t>(t) * a.nblk] = lds[t];
  }
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

// Raster work items: tile t's list is cut into max(1, ceil(L / kItemSplats))
// items, so no single workgroup carries a tile many times heavier than the
// mean.  items[t] receives the count here and its exclusive prefix after the
// scan; items[total_tiles] ends up holding the number of items.
__global__ __launch_bounds__(256) void make_items(const DevCamera* cams, int32_t nv, const uint32_t* hist,
                                                  int32_t nblk, int64_t capacity, int64_t total_tiles,
                                                  uint32_t* items) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t > total_tiles) return;
  if (t == total_tiles) {
    items[t] = 0u;
    return;
  }
  int v = 0;
  while (v + 1 < nv && cams[v + 1].tile_base <= t) ++v;
  const int64_t hb = cams[v].hist_base + (t - cams[v].tile_base) * nblk;
  const uint64_t cap = static_cast<uint64_t>(capacity);
  uint64_t s = hist[hb], e = hist[hb + nblk];
  s = s < cap ? s : cap;
  e = e < cap ? e : cap;
  const uint64_t len = e > s ? e - s : 0;
  items[t] = static_cast<uint32_t>(len == 0 ? 1 : (len + kItemSplats - 1) / kItemSplats);
}

}  // namespace

hipError_t launch_bin(const Layout& L, void* ws, void* pairs, int64_t capacity, hipStream_t st) {
  DevFlags* flags = at<DevFlags>(ws, L.off_flags);
  uint32_t* hist = at<uint32_t>(ws, L.off_hist);
  uint32_t* parts = at<uint32_t>(ws, L.off_scan);
  uint32_t* goff = at<uint32_t>(ws, L.off_goff);
  const int64_t len = L.hist_len + 1;  // trailing entry becomes the total
  const PairView pv = pair_view(pairs, capacity);

  BinArgs a;
  a.cams = at<DevCamera>(ws, L.off_cams);
  a.rect = at<uint2>(ws, L.off_rect);
  a.hist = hist;
  a.goff = goff;
  a.ids = pv.ids;
  a.slot = pv.slot;
  a.n = L.n;
  a.capacity = capacity;
  a.nblk = L.nblk;
  // whole tile rows per LDS chunk, at most kTileChunk tiles
  a.rows_per_chunk = kTileChunk / L.max_tiles_x;
  if (a.rows_per_chunk < 1) return hipErrorInvalidValue;
  const int nchunks = (L.max_tiles_y + a.rows_per_chunk - 1) / a.rows_per_chunk;
  const size_t lds = static_cast<size_t>(a.rows_per_chunk) * L.max_tiles_x * sizeof(uint32_t);
  const dim3 grid(static_cast<unsigned>(L.nblk), static_cast<unsigned>(nchunks), static_cast<unsigned>(L.nv));

  hipError_t e = launch_fill_zero(hist + L.hist_len, sizeof(uint32_t), st);
  if (e != hipSuccess) return e;
  // split-tile accumulator of the forward raster starts at zero
  e = launch_fill_zero(at<float>(ws, L.off_acc), sizeof(float) * 4 * L.total_pixels, st);
  if (e != hipSuccess) return e;
  bin_pass<false><<<grid, kBinThreads, lds, st>>>(a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Gaussian-major pair offsets (exclusive scan of the rectangle sizes)
  {
    const int64_t slots = L.n * L.nv;
    const int64_t glen = slots + 1;
    gauss_counts<<<static_cast<unsigned>((glen + 255) / 256), 256, 0, st>>>(a.rect, slots, goff);
    const unsigned gparts = static_cast<unsigned>((glen + kScanItems - 1) / kScanItems);
    scan_reduce<<<gparts, 256, 0, st>>>(goff, glen, parts);
    scan_parts<<<1, 1024, 0, st>>>(parts, gparts, nullptr, 0);
    scan_apply<<<gparts, 256, 0, st>>>(goff, glen, parts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const unsigned nparts = static_cast<unsigned>((len + kScanItems - 1) / kScanItems);
  scan_reduce<<<nparts, 256, 0, st>>>(hist, len, parts);
  scan_parts<<<1, 1024, 0, st>>>(parts, nparts, flags, capacity);
  scan_apply<<<nparts, 256, 0, st>>>(hist, len, parts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  bin_pass<true><<<grid, kBinThreads, lds, st>>>(a);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  // raster work items per tile, then their exclusive prefix
  uint32_t* items = at<uint32_t>(ws, L.off_items);
  const int64_t ilen = L.total_tiles + 1;
  make_items<<<static_cast<unsigned>((ilen + 255) / 256), 256, 0, st>>>(a.cams, L.nv, hist, L.nblk, capacity,
                                                                       L.total_tiles, items);
  const unsigned iparts = static_cast<unsigned>((ilen + kScanItems - 1) / kScanItems);
  scan_reduce<<<iparts, 256, 0, st>>>(items, ilen, parts);
  scan_parts<<<1, 1024, 0, st>>>(parts, iparts, nullptr, 0);
  scan_apply<<<iparts, 256, 0, st>>>(items, ilen, parts);
  return hipGetLastError();
}

}  // namespace wsr
