// Step a6 of the WSR path: per-tile lists of Gaussian ids with no depth key.
// Eq. 7 is a commutative sum (Sec. 4.2), so only membership matters; this is
// the step that replaces the per-tile depth sort of 3DGS (Sec. 4.1).
//
// A counting sort by tile built from LDS histograms, with no global atomics:
//   1. bin_pass<count>: block (b, z, v) takes Gaussians [b*kBinChunk, ...) of
//      view v and counts their (tile, Gaussian) pairs into an LDS histogram
//      of the tile rows of chunk z, written contiguously as row b of the
//      block-major count matrix M[v][b][tile].
//   2. column_scan_wide: each tile's column of M becomes exclusive prefixes
//      over the blocks, and the tile's total; tile_scan_single scans the
//      totals into the start of every tile's list (tile_start).
//   3. bin_pass<scatter>: the same blocks re-expand their pairs and place
//      each pair's entry (Gaussian id, Gaussian-major slot, see below) at
//      tile_start[t] + M[v][b][t] + the pair's stable rank in the block.
// Pairs are expanded load-balanced: per round of 256 Gaussians a block-wide
// scan of the pair counts lets every thread take every 256th pair, so one
// huge splat does not serialise on one thread.  The scatter is stable: every
// tile's list holds its Gaussian ids in increasing order, whatever the
// timing of the run.  Eq. 7 does not need an order, but the float sums of
// the raster stages follow the list order, so a fixed order makes the whole
// path reproducible bit for bit.
//
// The same step also lays out the backward's per-pair scratch: every
// (view, Gaussian) gets a contiguous range of "Gaussian-major" slots, one per
// tile of its rectangle in row-major order.  Its first slot, goff, is the
// exclusive scan of the rectangle sizes in (view, Gaussian) order, formed by
// the same passes: the counting pass's first band also sums each block's
// rectangle sizes, scan_parts scans those block sums, and the scatter pass's
// first band writes goff.  The raster work items that split long tile lists
// come from tile_scan_single.
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
  uint2* ent;                  // list entries (id, Gaussian-major slot)
  int64_t n;
  int64_t capacity;
  int32_t rows_per_chunk;
  int32_t nblk;                // blocks per view
  uint32_t* parts;             // per (view, block): sum of the rectangle sizes, then its exclusive scan
  uint32_t* goff;              // Gaussian-major first slot of every (view, Gaussian)
};

template <bool SCATTER>
__global__ __launch_bounds__(kBinThreads) void bin_pass(BinArgs a) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t s_off[kBinThreads];
  __shared__ uint32_t s_x0[kBinThreads], s_w[kBinThreads], s_y0[kBinThreads];
  __shared__ uint32_t s_gadj[kBinThreads];  // scatter: goff - (y0 w + x0), mod 2^32
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
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  // bits of a chunk-local tile index
  const int tbits = chunk_tiles > 1 ? 32 - __clz(static_cast<uint32_t>(chunk_tiles - 1)) : 1;
  const int64_t part = static_cast<int64_t>(v) * a.nblk + b;
  // running Gaussian-major offset of this block (counting pass: from 0, for
  // the block's sum; scatter pass: from the block's scanned offset)
  uint32_t gcarry = SCATTER ? a.parts[part] : 0u;
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
    if (SCATTER || z == 0) {
      // this (view, Gaussian)'s whole rectangle: its run of Gaussian-major
      // slots (counting pass, first band: the block's sum; scatter pass:
      // goff, stored by the first band, and each pair's slot)
      uint32_t full = 0, gadj = 0;
      if (i < g1) {
        const uint2 r = rect[i];
        const uint32_t rx0 = r.x & 0xffffu, rx1 = r.x >> 16, ry0r = r.y & 0xffffu, ry1r = r.y >> 16;
        full = (rx1 > rx0 && ry1r > ry0r) ? (rx1 - rx0) * (ry1r - ry0r) : 0u;
        gadj = 0u - (ry0r * (rx1 - rx0) + rx0);
      }
      uint32_t ftot;
      const uint32_t fex = block_scan_256(full, s_scan, &ftot);
      if (SCATTER) {
        s_gadj[threadIdx.x] = gcarry + fex + gadj;  // slot of tile (tx, ty): this + ty w + tx
        if (z == 0 && i < g1) a.goff[static_cast<int64_t>(v) * a.n + i] = gcarry + fex;
      }
      gcarry += ftot;
    }
    uint32_t total;
    const uint32_t off = block_scan_256(cnt, s_scan, &total);
    s_off[threadIdx.x] = off;
    s_x0[threadIdx.x] = x0;
    s_w[threadIdx.x] = w;
    s_y0[threadIdx.x] = y0;
    __syncthreads();
    // pairs p0 .. p0 + 255 of the round, in Gaussian-major order (a
    // Gaussian's tiles row-major), one per thread
    for (uint32_t p0 = 0; p0 < total; p0 += kBinThreads) {
      const uint32_t p = p0 + threadIdx.x;
      const bool valid = p < total;
      uint32_t t = 0, pslot = 0;
      int lo = 0;
      if (valid) {
        // largest g with s_off[g] <= p (it has a non-zero count)
        int hi = kBinThreads - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= p) lo = mid; else hi = mid - 1;
        }
        const uint32_t local = p - s_off[lo];
        const uint32_t ww = s_w[lo];
        const uint32_t ty = s_y0[lo] + local / ww;
        const uint32_t tx = s_x0[lo] + local % ww;
        t = (ty - ry0) * tiles_x + tx;
        if (SCATTER) pslot = s_gadj[lo] + ty * ww + tx;  // the pair's Gaussian-major slot
      }
      if (!SCATTER) {
        if (valid) atomicAdd(&lds[t], 1u);
        continue;
      }
      // Stable rank: the lanes of this wave holding the same tile are those
      // that agree with this lane on every bit of the tile index (one ballot
      // per bit); among them, lower lanes hold earlier pairs.
      const uint64_t vmask = __ballot(valid);
      uint64_t peers = vmask;
      for (int k = 0; k < tbits; ++k) {
        const bool bit = ((t >> k) & 1u) != 0u;
        const uint64_t bm = __ballot(valid && bit);
        if (bm != 0ull && bm != vmask) peers &= bit ? bm : ~bm;
      }
      const uint32_t rank = static_cast<uint32_t>(__popcll(peers & ((1ull << lane) - 1ull)));
      const uint32_t grp = static_cast<uint32_t>(__popcll(peers));
      const bool last = (peers >> lane) == 1ull;  // highest lane of its group
      // The waves place their pairs in turn (wave order is pair order): each
      // reads its tiles' cursors, and the last lane of a group advances its
      // tile's cursor past the group.
#pragma unroll
      for (int turn = 0; turn < kBinThreads / kWave; ++turn) {
        if (wv == turn && valid) {
          const uint32_t start = lds[t];
          const uint32_t pos = start + rank;
          if (pos < a.capacity)
            a.ent[pos] = make_uint2(static_cast<uint32_t>(base + lo), pslot);
          if (last) lds[t] = start + grp;
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
  if (!SCATTER) {
    for (int t = threadIdx.x; t < chunk_tiles; t += kBinThreads) row[t] = lds[t];
    if (z == 0 && threadIdx.x == 0) a.parts[part] = gcarry;
  }
}

// Column prefixes of the count matrix, 16 waves per 64 tiles: lane = tile (coalesced
// rows of the block-major matrix), wave w takes the w-th sixteenth of the
// blocks.  Pass 1 sums each wave's share, the waves' bases follow from LDS,
// pass 2 rewrites the share as exclusive prefixes.  Sixteen times the loads
// in flight of one thread per tile.
constexpr int kColWaves = 16;
__global__ __launch_bounds__(kColWaves * kWave) void column_scan_wide(const DevCamera* cams, int32_t nv,
                                                                      int32_t nblk, int64_t total_tiles,
                                                                      uint32_t* hist, uint32_t* tile_start) {
  __shared__ uint32_t s_sum[kColWaves][kWave];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWave + lane;
  const bool ok = t < total_tiles;
  uint32_t* col = hist;
  int64_t tiles_v = 0;
  if (ok) {
    int v = 0;
    while (v + 1 < nv && cams[v + 1].tile_base <= t) ++v;
    const DevCamera& cam = cams[v];
    tiles_v = static_cast<int64_t>(cam.tiles_x) * cam.tiles_y;
    col = hist + cam.hist_base + (t - cam.tile_base);
  }
  const int b0 = static_cast<int>(static_cast<int64_t>(nblk) * wv / kColWaves);
  const int b1 = static_cast<int>(static_cast<int64_t>(nblk) * (wv + 1) / kColWaves);
  uint32_t sum = 0;
  if (ok)
    for (int b = b0; b < b1; ++b) sum += col[b * tiles_v];
  s_sum[wv][lane] = sum;
  __syncthreads();
  uint32_t run = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kColWaves; ++w) {
    const uint32_t x = s_sum[w][lane];
    if (w < wv) run += x;
    total += x;
  }
  if (ok) {
    for (int b = b0; b < b1; ++b) {
      const uint32_t c = col[b * tiles_v];
      col[b * tiles_v] = run;
      run += c;
    }
    if (wv == 0) tile_start[t] = total;
  }
  if (wv == 0 && t == total_tiles) tile_start[t] = 0u;
}

// Exclusive scan over a 1024-thread block of one value per thread; *total
// receives the block sum.  `sh` needs 16 words.
__device__ inline uint32_t block_scan_1024(uint32_t v, uint32_t* sh, uint32_t* total) {
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
  for (int k = 0; k < 16; ++k) {
    const uint32_t x = sh[k];
    if (k < wv) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// One workgroup, after the column prefixes: the exclusive scan of the tile
// totals in place (tile_start; 64-bit running total, so a pair count beyond
// 32 bits is detected), the overflow flags, the raster work items --
// max(1, ceil(list length / kItemSplats)) per tile -- with their exclusive
// scan (items[total_tiles] = number of items), and their dispatch order.
// One pass over the tiles forms the starts, the item counts and the order
// histogram; a second places the tiles in the order.
constexpr int kTileScanThreads = 1024;
constexpr int kTileScanPer = 8;
constexpr int kOrderBuckets = kItemSplats / 32 + 1;

// A tile's list length with both ends capped at the pair capacity.
__device__ __forceinline__ uint64_t capped_len(uint64_t a, uint64_t e, uint64_t cap) {
  a = a < cap ? a : cap;
  e = e < cap ? e : cap;
  return e > a ? e - a : 0;
}

// Bucket of a tile in the dispatch order, from its (capped) list length:
// longest last work item first.
__device__ __forceinline__ int order_bucket(uint64_t l) {
  const uint64_t last = l == 0 ? 0 : l - ((l - 1) / kItemSplats) * kItemSplats;  // in [1, kItemSplats]
  return kOrderBuckets - 1 - static_cast<int>(last / 32);
}

// Dispatch order of the work items.  Items that hold a full kItemSplats
// splats run first (in tile order: dispatch slot i < F, F the number of such
// items, is tile t's full item i - (items[t] - t)); then every tile's last
// item, longest first: tile_order lists the tiles by the length of that
// item, counting-sorted in buckets of 32 splats.  Heavy items start early,
// so the launch ends on short ones instead of waiting for a late heavy one.
// Only the order of execution changes (within a bucket it varies from run
// to run): every item writes the same outputs.
__global__ __launch_bounds__(kTileScanThreads) void tile_scan_single(uint32_t* tile_start, int64_t total_tiles,
                                                                     uint32_t* items, uint32_t* tile_order,
                                                                     DevFlags* flags, int64_t capacity) {
  __shared__ uint32_t sh[16];
  __shared__ uint32_t bucket[kOrderBuckets];
  for (int k = threadIdx.x; k < kOrderBuckets; k += kTileScanThreads) bucket[k] = 0u;
  const int64_t len = total_tiles + 1;
  const uint64_t cap = static_cast<uint64_t>(capacity);
  constexpr int64_t kChunk = static_cast<int64_t>(kTileScanThreads) * kTileScanPer;
  uint64_t carry = 0;
  uint32_t icarry = 0;
  for (int64_t c0 = 0; c0 < len; c0 += kChunk) {
    const int64_t base = c0 + static_cast<int64_t>(threadIdx.x) * kTileScanPer;
    uint32_t vals[kTileScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kTileScanPer; ++k) {
      vals[k] = base + k < len ? tile_start[base + k] : 0u;
      s += vals[k];
    }
    uint32_t tot;
    uint64_t run = carry + block_scan_1024(s, sh, &tot);  // (its first barrier also orders the bucket clear)
    uint32_t icnt[kTileScanPer];
    uint32_t is = 0;
#pragma unroll
    for (int k = 0; k < kTileScanPer; ++k) {
      const int64_t t = base + k;
      if (t < len) tile_start[t] = static_cast<uint32_t>(run);
      icnt[k] = 0u;
      if (t < total_tiles) {
        // from the 32-bit starts as stored, which the placement pass reads
        const uint64_t l = capped_len(static_cast<uint32_t>(run), static_cast<uint32_t>(run + vals[k]), cap);
        icnt[k] = static_cast<uint32_t>(l == 0 ? 1 : (l + kItemSplats - 1) / kItemSplats);
        atomicAdd(&bucket[order_bucket(l)], 1u);
      }
      is += icnt[k];
      run += vals[k];
    }
    carry += tot;
    uint32_t itot;
    uint32_t irun = icarry + block_scan_1024(is, sh, &itot);
#pragma unroll
    for (int k = 0; k < kTileScanPer; ++k) {
      if (base + k < len) items[base + k] = irun;
      irun += icnt[k];
    }
    icarry += itot;
  }
  if (threadIdx.x == 0) {
    flags->total_pairs = carry;
    flags->wrapped = carry > 0xffffffffull ? 1u : 0u;
    flags->overflow = (carry > static_cast<uint64_t>(capacity) || carry > 0xffffffffull) ? 1u : 0u;
    flags->sort_overflow = 0u;
    flags->cull_masks = 0u;  // new lists: no culling masks yet
    uint32_t r = 0;
    for (int k = 0; k < kOrderBuckets; ++k) {
      const uint32_t c = bucket[k];
      bucket[k] = r;
      r += c;
    }
  }
  __syncthreads();  // the starts of every tile and the bucket offsets are in place
  for (int64_t t = threadIdx.x; t < total_tiles; t += kTileScanThreads)
    tile_order[atomicAdd(&bucket[order_bucket(capped_len(tile_start[t], tile_start[t + 1], cap))], 1u)] =
        static_cast<uint32_t>(t);
}

// Exclusive scan (in place) of the per-(view, block) rectangle sums, in
// (view, block) order, i.e. (view, Gaussian) order; the grand total goes to
// *total (goff's closing entry).
__global__ __launch_bounds__(1024) void scan_parts(uint32_t* parts, int64_t nparts, uint32_t* total) {
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
  if (threadIdx.x == 0) *total = static_cast<uint32_t>(carry);
}

}  // namespace

hipError_t launch_bin(const Layout& L, void* ws, void* pairs, int64_t capacity, hipStream_t st) {
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
  a.ent = pv.ent;
  a.n = L.n;
  a.capacity = capacity;
  a.nblk = L.nblk;
  a.parts = parts;
  a.goff = goff;
  // whole tile rows per LDS chunk, at most kTileChunk tiles, and at least
  // kBinBands chunks of rows: each block then expands only the pairs of its
  // band, and the four times more blocks keep more of the chip busy (binning
  // 0.254 -> 0.214 ms at 1 M Gaussians / 1080p)
  constexpr int kBinBands = 4;
  if (kTileChunk / L.max_tiles_x < 1) return hipErrorInvalidValue;
  a.rows_per_chunk = min(kTileChunk / L.max_tiles_x, (L.max_tiles_y + kBinBands - 1) / kBinBands);
  if (a.rows_per_chunk < 1) a.rows_per_chunk = 1;
  const int nchunks = (L.max_tiles_y + a.rows_per_chunk - 1) / a.rows_per_chunk;
  const size_t lds = static_cast<size_t>(a.rows_per_chunk) * L.max_tiles_x * sizeof(uint32_t);
  const dim3 grid(static_cast<unsigned>(L.nblk), static_cast<unsigned>(nchunks), static_cast<unsigned>(L.nv));

  hipError_t e;
  bin_pass<false><<<grid, kBinThreads, lds, st>>>(a);
  column_scan_wide<<<static_cast<unsigned>((L.total_tiles + 1 + kWave - 1) / kWave), kColWaves * kWave, 0, st>>>(
      a.cams, L.nv, L.nblk, L.total_tiles, hist, tstart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // tile starts, overflow flags and raster work items in one workgroup
  tile_scan_single<<<1, kTileScanThreads, 0, st>>>(tstart, L.total_tiles, items,
                                                   at<uint32_t>(ws, L.off_torder), flags, capacity);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Gaussian-major offsets of the blocks (the counting pass summed each
  // block's rectangle sizes); the scatter pass writes goff
  scan_parts<<<1, 1024, 0, st>>>(parts, static_cast<int64_t>(L.nv) * L.nblk, goff + L.n * L.nv);
  bin_pass<true><<<grid, kBinThreads, lds, st>>>(a);
  return hipGetLastError();
}

}  // namespace wsr
