// Steps a7 and a8 of the WSR path: the per-pixel weighted sums of Sec. 4.2,
// Eq. 7, and their gradient.
//
//   forward:  N = c_B w_B + sum_i c_i a_i,  D = w_B + sum_i a_i,  C = N / D
//             a_i = amp_i exp(-q_i / 2) for q_i <= tau   (amp_i = u_i w(d_i))
//   backward: per pixel gbar = dL/dC / D and s = gbar . C; per pair
//             dL/da = gbar . c_i - s, then the chain to (mu, conic, c, amp).
//
// One workgroup per work item (at most kItemSplats splats of one tile's list); the
// items are dispatched longest first (the full ones, then the tiles' last
// items by decreasing length; see tile_scan_single), so that the launch ends
// on short items.
// Each wave owns an 8x8 pixel block of the tile.  Per batch the group stages
// splat records into LDS; each wave then keeps only the splats whose support
// reaches its own block (support box, then the exact minimum of q over the
// block; wave ballot + compaction into an LDS list).  In the forward every
// lane evaluates its pixel against that list with FP32 register
// accumulation; in the backward every lane takes one splat of the list and
// walks the block.  The sums are commutative, so the list order does not
// matter, and no per-pair data is stored between forward and backward: the
// backward recomputes every pair.
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "wsr_internal.h"

namespace wsr {
namespace {

// Every wave owns an 8x8 pixel block of the tile (one pixel per lane): tile 8
// is one wave, tile 16 four, tile 32 sixteen.  Up to 256 records are staged
// per batch.
template <int T>
struct TileGeom {
  static constexpr int kSub = 8;                       // wave block edge
  static constexpr int kWaves = (T / 8) * (T / 8);
  static constexpr int kThreads = kWaves * kWave;
  static constexpr int kBatch = kThreads < 256 ? kThreads : 256;
  static_assert(kBatch <= 256, "the backward's lists hold 8-bit record indices");
};

// A record as staged in LDS for one tile (48 bytes; stage_and_cull builds it
// from the projected record):
//   r0 = (mx, my, A, B2)   centre relative to the tile's centre; conic
//                          (A, B2 = 2B, C) times log2(e) / 2
//   r1 = (C, amp, c0, c1)  colour (times amp in the forward)
//   r2 = (c2, ext | cut, u, 0)  support half-extents (two halves), or with
//                          the early-out the record's own cutoff times
//                          log2(e) / 2; u = the opacity, used by OIT only
// The tile-relative centre is (integer origin - tile centre) + fractional
// centre: the difference is exact, the sum rounds once (to within 2^-24 of
// its magnitude, which is at most the pixel's distance plus half the tile
// size).  Pixel centres relative to the tile centre are exact, so dx and dy
// round once more.  With the conic scaled, the form below is q log2(e) / 2, the
// falloff exp(-q / 2) is one hardware exp2 of its negation, and every cutoff
// it is compared with (tau, a record's own cutoff) carries the same factor.
struct StagedRec {
  float4 r0, r1, r2;
};
static_assert(sizeof(StagedRec) == 48, "staged record layout");

constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
constexpr float kTwoLn2 = 1.38629436111989061f;     // its inverse

// The support predicate and the Gaussian falloff.  Forward and backward
// evaluate q with exactly this sequence of float operations (the backward
// hoists the row-constant products B2*dy and (C*dy)*dy, which does not change
// their values), so both take the same support decision for every pair.
// Different tile sizes round the tile-relative centre differently, so they
// can disagree on a pair within that rounding of the cutoff.
__device__ __forceinline__ float quad_form(float A, float B2dy, float Cdy2, float dx) {
  return fmaf(fmaf(A, dx, B2dy), dx, Cdy2);
}

// px, py: the pixel centre relative to the tile's centre
__device__ __forceinline__ float pair_q(const StagedRec& r, float px, float py) {
  const float dx = px - r.r0.x;
  const float dy = py - r.r0.y;
  return quad_form(r.r0.z, r.r0.w * dy, (r.r1.x * dy) * dy, dx);
}

// exp(-q/2) from the scaled form q log2(e) / 2
__device__ __forceinline__ float falloff(float qs) { return __builtin_amdgcn_exp2f(-qs); }

__device__ __forceinline__ float2 rec_extent(const StagedRec& r) {
  const uint32_t e = __float_as_uint(r.r2.y);
  const _Float16 ex = __builtin_bit_cast(_Float16, static_cast<uint16_t>(e & 0xffffu));
  const _Float16 ey = __builtin_bit_cast(_Float16, static_cast<uint16_t>(e >> 16));
  return make_float2(static_cast<float>(ex), static_cast<float>(ey));
}

// Does the splat's support reach the wave block whose pixel centres span
// [bx, bx + sub1] x [by, by + sub1] (relative to the tile's centre)?  First
// the (conservative) support box; then, unless the conic is badly
// conditioned, the exact minimum of q over
// the block (the unconstrained minimum is the centre; otherwise the minimum
// lies on an edge, at the clamped 1D minimiser of that edge) against tau with
// a margin far above the float error of q.  For needle-like splats
// (eigenvalue ratio above ~100) float q loses digits to cancellation, so the
// box decision is kept.
//
// With CUT (the opacity early-out) the record's fourth word is the splat's
// own cutoff instead of the half-extents, which are then derived from the
// conic: the extents of q <= cut are sqrt(cut C / det) and sqrt(cut A / det),
// with det = A C - B^2 formed by Kahan's algorithm (B^2 split exactly with an
// FMA) so that it stays accurate for needle-like conics.
template <bool CUT>
__device__ __forceinline__ bool block_hits(const StagedRec& r, float bx, float by, float sub1, float tau_in) {
  float2 e;
  float tau = tau_in;
  if (CUT) {
    tau = r.r2.y;
    const float A = r.r0.z, B = 0.5f * r.r0.w, C = r.r1.x;
    const float bb = B * B;
    const float det = fmaf(A, C, -bb) - fmaf(B, B, -bb);
    const float s = det > 0.f ? tau * __builtin_amdgcn_rcpf(det) : __builtin_inff();
    e = make_float2(sqrtf(s * C) * 1.0001f, sqrtf(s * A) * 1.0001f);
  } else {
    e = rec_extent(r);
  }
  const float mx = r.r0.x, my = r.r0.y;
  const float sx = 1e-3f * fabsf(mx) + 1e-2f, sy = 1e-3f * fabsf(my) + 1e-2f;  // rounding slack
  if (!((mx + e.x + sx >= bx) && (mx - e.x - sx <= bx + sub1) && (my + e.y + sy >= by) &&
        (my - e.y - sy <= by + sub1)))
    return false;
  const float A = r.r0.z, B = 0.5f * r.r0.w, C = r.r1.x;
  const float tr = A + C, det = A * C - B * B;
  if (!(tr * tr <= 102.f * det)) return true;
  // block corners relative to the centre
  const float x0 = bx - mx, x1 = (bx + sub1) - mx;
  const float y0 = by - my, y1 = (by + sub1) - my;
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
  // hardware reciprocals (within 1 ulp): they only place the edge minimisers,
  // whose error changes q there by a second-order amount far inside the margin
  const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
  float qmin = 3.0e38f;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float dy = k ? y1 : y0;
    const float dx = fminf(fmaxf(-B * dy * iA, x0), x1);
    qmin = fminf(qmin, A * dx * dx + 2.f * B * dx * dy + C * dy * dy);
    const float ex2 = k ? x1 : x0;
    const float ey2 = fminf(fmaxf(-B * ex2 * iC, y0), y1);
    qmin = fminf(qmin, A * ex2 * ex2 + 2.f * B * ex2 * ey2 + C * ey2 * ey2);
  }
  return qmin <= tau * 1.002f + 1e-3f;
}

struct RasterArgs {
  const DevCamera* cams;
  const DevSplat* rec;
  const uint32_t* tile_start;  // start of every tile's id list
  const uint2* ent;       // list entries (Gaussian id, Gaussian-major slot)
  int64_t n;
  int64_t capacity;
  int32_t nv;
  float tau;              // support cutoff, times log2(e) / 2 like the staged conic
  int32_t unnormalised;   // write the raw sums (no background, no division)
  const float* globals;
  // forward outputs
  float* out_rgb;
  float* out_den;
  int32_t* out_count;
  // backward inputs / outputs
  const float* dL_drgb;
  const float* rgb;
  const float* den;
  float3* part;           // per-pair partial 2D gradients, 3 float3 per slot
  float* tilepart;
  // work items (see tile_scan_single); the split-tile partial sums of the
  // forward: item 0 of a split tile in the per-pixel accumulator, item k > 0
  // of the tile with first item i0 at slot i0 - tile + k - 1 of split4 (and
  // splitlog for Eq. 2's coverage), [split_slots][T * T]
  const uint32_t* items;
  const uint32_t* tile_order;  // dispatch order of the tiles' last items
  int64_t total_tiles;
  float* acc;
  float4* split4;
  float* splitlog;
  int64_t split_slots;
  // OIT (Eq. 2): per pixel (weighted average, coverage P) from the forward,
  // the split-tile accumulator of ln P and the per-pair partial dL/du
  float4* oit;
  float* acclog;
  float* du;
  // persistent launches: the counter the workgroups take work items from
  // (zeroed before the launch); null for one workgroup per work item
  uint32_t* queue;
  // culling masks (see cull_mask_word), or null where the pair buffer has no
  // room for them; flags->cull_masks says whether they hold the current
  // lists' masks
  uint64_t* masks;
  DevFlags* flags;
};

// A persistent workgroup's next work item: the next unclaimed one, taken
// from the counter by thread 0 and shared through LDS.
__device__ __forceinline__ uint32_t claim_item(const RasterArgs& a, uint32_t* s_item) {
  __syncthreads();  // every thread has read the previous item
  if (threadIdx.x == 0) *s_item = atomicAdd(a.queue, 1u);
  __syncthreads();
  return *s_item;
}

__device__ __forceinline__ int find_view(const DevCamera* cams, int nv, int tile) {
  int v = 0;
  while (v + 1 < nv && cams[v + 1].tile_base <= tile) ++v;
  return v;
}

// Common set-up of one work item: its tile (view, tile coordinates), the
// sub-range [start, end) of the tile's id list it covers, and this lane's
// pixels.
template <int T>
struct TileCtx {
  int v, tx, ty;
  int64_t tile;
  int64_t n;
  uint32_t start, end;
  uint32_t list0;                 // first list position of the tile (capped at the capacity)
  uint32_t k, nk;                 // item index within the tile, items of the tile
  int wave, lane;
  int bx0, by0;                   // first pixel of this wave's block
  int px, py;                     // this lane's pixel
  int fx0, fy0;                   // frame origin of the staged centres: the tile's centre
};

// The culling masks: wave w's 64-bit ballot for the 64-entry group g of tile
// t's list (entries list0 + 64 g ...) is word (list0 / 64 + t + g) W + w, W the
// waves of a tile.  A tile of l entries has ceil(l / 64) groups and the next
// tile's first group is at least floor((list0 + l) / 64) + t + 1, so the
// tiles' words never overlap; all of them lie below
// (ceil(capacity / 64) + tiles + 2) W.
template <int T>
__device__ __forceinline__ int64_t cull_mask_word(const TileCtx<T>& c, uint32_t pos) {
  constexpr int W = TileGeom<T>::kWaves;
  const int64_t g = static_cast<int64_t>(c.list0 >> 6) + c.tile + ((pos - c.list0) >> 6);
  return g * W + c.wave;
}

template <int T>
__device__ __forceinline__ void tile_setup(const RasterArgs& a, uint32_t item, TileCtx<T>& c, const DevCamera*& cam) {
  using G = TileGeom<T>;
  // dispatch slot -> (tile, item within the tile), in the order the binning
  // laid out: first the full items, tile by tile, then the tiles' last items
  // in tile_order
  const uint32_t nfull = a.items[a.total_tiles] - static_cast<uint32_t>(a.total_tiles);
  int64_t lo = 0;
  if (item < nfull) {
    // largest tile t with items[t] - t <= item (nondecreasing in t)
    int64_t hi = a.total_tiles - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (static_cast<int64_t>(a.items[mid]) - mid <= static_cast<int64_t>(item)) lo = mid; else hi = mid - 1;
    }
    c.k = item - (a.items[lo] - static_cast<uint32_t>(lo));
  } else {
    lo = a.tile_order[item - nfull];
    c.k = a.items[lo + 1] - a.items[lo] - 1;
  }
  c.tile = lo;
  c.nk = a.items[lo + 1] - a.items[lo];
  const int tile = static_cast<int>(lo);
  c.v = find_view(a.cams, a.nv, tile);
  cam = &a.cams[c.v];
  const int local = tile - cam->tile_base;
  c.tx = local % cam->tiles_x;
  c.ty = local / cam->tiles_x;
  c.n = a.n;
  const uint64_t cap = static_cast<uint64_t>(a.capacity);
  uint64_t s = a.tile_start[lo], e = a.tile_start[lo + 1];
  s = s < cap ? s : cap;
  e = e < cap ? e : cap;
  if (e < s) e = s;
  c.list0 = static_cast<uint32_t>(s);
  const uint64_t ss = s + static_cast<uint64_t>(c.k) * kItemSplats;
  const uint64_t ee = ss + kItemSplats;
  c.start = static_cast<uint32_t>(ss < e ? ss : e);
  c.end = static_cast<uint32_t>(ee < e ? ee : e);
  c.wave = threadIdx.x / kWave;
  c.lane = threadIdx.x % kWave;
  c.bx0 = c.tx * T + (c.wave % (T / 8)) * G::kSub;
  c.by0 = c.ty * T + (c.wave / (T / 8)) * G::kSub;
  c.fx0 = c.tx * T + T / 2;
  c.fy0 = c.ty * T + T / 2;
  c.px = c.bx0 + (c.lane & 7);
  c.py = c.by0 + (c.lane >> 3);
}

// Stage one batch of records into LDS (as StagedRec) and build this wave's
// culled list.  Returns the list length.  With PREMUL (the forward) the
// staged colour is premultiplied by the amplitude, so a pair adds G (amp c)
// and G amp.  The list holds staged-record indices (uint8_t) or, as uint32_t,
// their byte offsets in s_rec, which the forward uses as LDS addresses
// directly.  With SLOTS (the backward), also the Gaussian-major slot of
// each staged (tile, splat) pair -- the Gaussian's first slot plus this
// tile's row-major index in its tile rectangle, the order in which binning
// enumerated its pairs -- and, per staged record, its position in this
// wave's list (0xffff if culled).
template <int T, int BATCH, bool SLOTS, bool CUT, bool OIT, bool PREMUL, typename LT>
__device__ __forceinline__ int stage_and_cull(const RasterArgs& a, const TileCtx<T>& c, uint32_t b,
                                              StagedRec* s_rec, uint32_t* s_slot, LT* s_list,
                                              uint16_t* s_pos, uint64_t* mask_out = nullptr,
                                              const uint64_t* mask_in = nullptr) {
  using G = TileGeom<T>;
  const float tox = static_cast<float>(c.fx0), toy = static_cast<float>(c.fy0);
  __syncthreads();  // previous batch fully consumed
  for (int q = threadIdx.x; q < BATCH; q += G::kThreads) {
    const uint32_t j = b + q;
    if (j < c.end) {
      const uint2 en = a.ent[j];  // (Gaussian id, the pair's Gaussian-major slot)
      const DevSplat* d = a.rec + static_cast<int64_t>(c.v) * c.n + en.x;
      const SplatRec s = d->s;  // (fx, fy, A, B2) (C, ox, oy, amp) (c0, c1, c2, ext | cut)
      const float amp = s.r1.w;
      float c0 = s.r2.x, c1 = s.r2.y, c2 = s.r2.z;
      if (PREMUL) {
        c0 *= amp;
        c1 *= amp;
        c2 *= amp;
      }
      StagedRec r;
      r.r0 = make_float4((s.r1.y - tox) + s.r0.x, (s.r1.z - toy) + s.r0.y, s.r0.z * kHalfLog2e,
                         s.r0.w * kHalfLog2e);
      r.r1 = make_float4(s.r1.x * kHalfLog2e, amp, c0, c1);
      // OIT: the opacity u rides in the record's third word
      r.r2 = make_float4(c2, CUT ? s.r2.w * kHalfLog2e : s.r2.w, OIT ? __uint_as_float(d->slot.w) : 0.f, 0.f);
      s_rec[q] = r;
      if (SLOTS) s_slot[q] = en.y;
    }
  }
  __syncthreads();
  const int cnt = static_cast<int>(min(static_cast<uint32_t>(BATCH), c.end - b));
  LT* list = s_list + c.wave * BATCH;
  int m = 0;
  const float bx = static_cast<float>(c.bx0 - c.fx0) + 0.5f, by = static_cast<float>(c.by0 - c.fy0) + 0.5f;
  for (int k0 = 0; k0 < cnt; k0 += kWave) {
    const int k = k0 + c.lane;
    bool hit;
    uint64_t mask;
    if (mask_in) {
      // the forward's ballot for these entries: the same test of the same
      // staged values (the staged colour aside), so the same lists
      mask = mask_in[cull_mask_word(c, b + k0)];
      hit = ((mask >> c.lane) & 1ull) != 0;
    } else {
      hit = k < cnt && block_hits<CUT>(s_rec[k], bx, by, static_cast<float>(G::kSub - 1), a.tau);
      mask = __ballot(hit);
      if (mask_out && c.lane == 0) mask_out[cull_mask_word(c, b + k0)] = mask;
    }
    const int pos = m + __popcll(mask & ((1ull << c.lane) - 1ull));
    if (hit) {
      if constexpr (sizeof(LT) == 8)
        list[pos] = LT{static_cast<uint32_t>(k * static_cast<int>(sizeof(StagedRec))), __float_as_uint(s_rec[k].r2.x)};
      else
        list[pos] = static_cast<LT>(sizeof(LT) == 1 ? k : k * static_cast<int>(sizeof(StagedRec)));
    }
    if (SLOTS && k < BATCH) s_pos[c.wave * BATCH + k] = hit ? static_cast<uint16_t>(pos) : 0xffffu;
    m += __popcll(mask);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return m;
}

// Eq. 7 for one pixel from its sums (or the raw sums in unnormalised mode).
__device__ __forceinline__ void write_pixel(const RasterArgs& a, int64_t pix, float nr, float ng, float nb,
                                            float dd) {
  if (a.unnormalised) {
    a.out_rgb[3 * pix] = nr;
    a.out_rgb[3 * pix + 1] = ng;
    a.out_rgb[3 * pix + 2] = nb;
    a.out_den[pix] = dd;
    return;
  }
  const float wbg = a.globals[2];
  const float bgr = a.globals[3], bgg = a.globals[4], bgb = a.globals[5];
  const float D = wbg + dd;
  const float Nr = fmaf(bgr, wbg, nr), Ng = fmaf(bgg, wbg, ng), Nb = fmaf(bgb, wbg, nb);
  float Cr = bgr, Cg = bgg, Cb = bgb;
  if (D != 0.f) {
    Cr = Nr / D;
    Cg = Ng / D;
    Cb = Nb / D;
  }
  a.out_rgb[3 * pix] = Cr;
  a.out_rgb[3 * pix + 1] = Cg;
  a.out_rgb[3 * pix + 2] = Cb;
  a.out_den[pix] = D;
}

// Eq. 2 for one pixel: C = P c_B + (1 - P) N / D (the average is 0 where
// D = 0); D goes to out_den and (N / D, P) to the workspace for the backward.
__device__ __forceinline__ void write_pixel_oit(const RasterArgs& a, int64_t pix, float nr, float ng, float nb,
                                                float dd, float P) {
  const float inv = dd != 0.f ? 1.f / dd : 0.f;
  const float ar = nr * inv, ag = ng * inv, ab = nb * inv;
  const float Q = 1.f - P;
  a.out_rgb[3 * pix] = fmaf(P, a.globals[3], Q * ar);
  a.out_rgb[3 * pix + 1] = fmaf(P, a.globals[4], Q * ag);
  a.out_rgb[3 * pix + 2] = fmaf(P, a.globals[5], Q * ab);
  a.out_den[pix] = dd;
  a.oit[pix] = make_float4(ar, ag, ab, P);
}

__device__ __forceinline__ const StagedRec& rec_at(const StagedRec* base, uint32_t off) {
  return *reinterpret_cast<const StagedRec*>(reinterpret_cast<const char*>(base) + off);
}

// The first two vectors of a staged record (centre, conic, amplitude and two
// premultiplied colours): with 8-byte list entries, whose second word holds
// the third colour, a forward step reads two 16-byte vectors per record.
struct StagedHead {
  float4 r0, r1;
};
__device__ __forceinline__ StagedHead head_at(const StagedRec* base, uint32_t off) {
  const StagedRec& r = rec_at(base, off);
  return StagedHead{r.r0, r.r1};
}

// List entry type of the forward: with the weighted sum of Eq. 7 (no
// per-splat cutoff, no opacity), (record byte offset, third premultiplied
// colour), so that one 16-byte read fetches two entries and a step reads
// 2.5 LDS vectors instead of 3.25; otherwise the byte offset alone.
template <bool CUT, bool OIT>
using FwdList = typename std::conditional<!CUT && !OIT, uint2, uint32_t>::type;

// The forward of one work item (tile_setup's c), S records staged per batch.
template <int T, int S, bool COUNT, bool CUT, bool OIT>
__device__ __forceinline__ void raster_fwd_item(const RasterArgs& a, const TileCtx<T>& c, const DevCamera* cam,
                                                StagedRec* s_rec, FwdList<CUT, OIT>* s_list) {
  using LT = FwdList<CUT, OIT>;
  float nr = 0.f, ng = 0.f, nb = 0.f, dd = 0.f;
  float cov = 1.f;  // OIT: prod (1 - alpha)
  int cntp = 0;
  // this lane's pixel centre relative to the tile's centre (exact)
  const float pcx = static_cast<float>(c.px - c.fx0) + 0.5f;
  const float pcy = static_cast<float>(c.py - c.fy0) + 0.5f;
  const float tau = a.tau;
  for (uint32_t b = c.start; b < c.end; b += S) {
    const int m = stage_and_cull<T, S, false, CUT, OIT, true, LT>(a, c, b, s_rec, nullptr, s_list, nullptr,
                                                                  a.masks);
    const LT* list = s_list + c.wave * S;
    // four splats per step: one read fetches their list entries and all four
    // records are requested before any arithmetic, so LDS latency is paid
    // once per four splats.  The staged colour carries the amplitude.
    auto accumulate = [&](const StagedRec& r) {
      const float q = pair_q(r, pcx, pcy);
      const float cut = CUT ? r.r2.y : tau;
      const float G = q <= cut ? falloff(q) : 0.f;
      nr = fmaf(G, r.r1.z, nr);
      ng = fmaf(G, r.r1.w, ng);
      nb = fmaf(G, r.r2.x, nb);
      dd = fmaf(G, r.r1.y, dd);
      if (OIT) cov *= 1.f - __builtin_amdgcn_fmed3f(r.r2.z * G, 0.f, 1.f);
      if (COUNT) cntp += q <= cut ? 1 : 0;
    };
    int i = 0;
    if constexpr (sizeof(LT) == 8) {
      // the same arithmetic as accumulate, with the third colour from the entry
      auto accumulate_head = [&](const StagedHead& r, float cb) {
        const float dx = pcx - r.r0.x;
        const float dy = pcy - r.r0.y;
        const float q = quad_form(r.r0.z, r.r0.w * dy, (r.r1.x * dy) * dy, dx);
        const float G = q <= tau ? falloff(q) : 0.f;
        nr = fmaf(G, r.r1.z, nr);
        ng = fmaf(G, r.r1.w, ng);
        nb = fmaf(G, cb, nb);
        dd = fmaf(G, r.r1.y, dd);
        if (COUNT) cntp += q <= tau ? 1 : 0;
      };
      for (; i + 4 <= m; i += 4) {
        const uint4 e01 = *reinterpret_cast<const uint4*>(list + i);
        const uint4 e23 = *reinterpret_cast<const uint4*>(list + i + 2);
        const StagedHead r0 = head_at(s_rec, e01.x);
        const StagedHead r1 = head_at(s_rec, e01.z);
        const StagedHead r2 = head_at(s_rec, e23.x);
        const StagedHead r3 = head_at(s_rec, e23.z);
        accumulate_head(r0, __uint_as_float(e01.y));
        accumulate_head(r1, __uint_as_float(e01.w));
        accumulate_head(r2, __uint_as_float(e23.y));
        accumulate_head(r3, __uint_as_float(e23.w));
      }
      for (; i < m; ++i) {
        const uint2 e = list[i];
        accumulate_head(head_at(s_rec, e.x), __uint_as_float(e.y));
      }
    } else {
      for (; i + 4 <= m; i += 4) {
        const uint4 o4 = *reinterpret_cast<const uint4*>(list + i);
        const StagedRec r0 = rec_at(s_rec, o4.x);
        const StagedRec r1 = rec_at(s_rec, o4.y);
        const StagedRec r2 = rec_at(s_rec, o4.z);
        const StagedRec r3 = rec_at(s_rec, o4.w);
        accumulate(r0);
        accumulate(r1);
        accumulate(r2);
        accumulate(r3);
      }
      for (; i < m; ++i) accumulate(rec_at(s_rec, list[i]));
    }
  }
  if (c.px >= cam->width || c.py >= cam->height) return;
  const int64_t pix = cam->pix_base + static_cast<int64_t>(c.py) * cam->width + c.px;
  if (COUNT) atomicAdd(a.out_count + pix, cntp);
  if (c.nk > 1) {
    // split tile: this item's partial sums, added in item order by
    // raster_fwd_finalize (the coverage products of the parts multiply, so
    // their logarithms add).  Item 0 stores into the per-pixel accumulator,
    // item k > 0 into its own slot of the split-tile partials.
    const float4 sums = make_float4(nr, ng, nb, dd);
    if (c.k == 0) {
      reinterpret_cast<float4*>(a.acc)[pix] = sums;
      if (OIT) a.acclog[pix] = __logf(cov);
    } else {
      const int64_t e = static_cast<int64_t>(a.items[c.tile]) - c.tile + c.k - 1;
      if (e < a.split_slots) {
        const int64_t q = e * (T * T) + (c.py - c.ty * T) * T + (c.px - c.tx * T);
        a.split4[q] = sums;
        if (OIT) a.splitlog[q] = __logf(cov);
      }
    }
    return;
  }
  if (OIT)
    write_pixel_oit(a, pix, nr, ng, nb, dd, cov);
  else
    write_pixel(a, pix, nr, ng, nb, dd);
}

// Forward.  Lists hold LDS byte offsets of the staged records.  S records
// are staged per batch.  A workgroup renders the work item of dispatch slot
// blockIdx.x (the grid covers them all), or, PERSIST, claims slots from a
// counter until none is left.
template <int T, int S, bool COUNT, bool CUT, bool OIT, bool PERSIST>
__global__ __launch_bounds__(TileGeom<T>::kThreads) void raster_fwd_kernel(RasterArgs a) {
  using G = TileGeom<T>;
  using LT = FwdList<CUT, OIT>;
  __shared__ StagedRec s_rec[S];
  __shared__ __align__(16) LT s_list[G::kWaves * S];
  __shared__ uint32_t s_item;
  // every work item stores its waves' culling masks (when there is room):
  // valid for the backward once this launch has finished
  if (blockIdx.x == 0 && threadIdx.x == 0) a.flags->cull_masks = a.masks ? (kCullMasks | (CUT ? 2u : 0u)) : 0u;
  const uint32_t n_items = a.items[a.total_tiles];
  uint32_t item = PERSIST ? claim_item(a, &s_item) : blockIdx.x;
  while (item < n_items) {
    TileCtx<T> c;
    const DevCamera* cam;
    tile_setup<T>(a, item, c, cam);
    raster_fwd_item<T, S, COUNT, CUT, OIT>(a, c, cam, s_rec, s_list);
    if (!PERSIST) break;
    item = claim_item(a, &s_item);
  }
}

// Normalisation of the tiles whose list was split over several work items:
// the items' partial sums are added in item order (item 0's from the
// per-pixel accumulator, the others' from their slots), so the image does
// not depend on the order in which the items ran.
template <int T, bool OIT>
__global__ __launch_bounds__(256) void raster_fwd_finalize(RasterArgs a) {
  const int64_t t = blockIdx.x;
  const uint32_t i0 = a.items[t], nk = a.items[t + 1] - i0;
  if (nk <= 1) return;
  const int tile = static_cast<int>(t);
  const int v = find_view(a.cams, a.nv, tile);
  const DevCamera& cam = a.cams[v];
  const int local = tile - cam.tile_base;
  const int tx = local % cam.tiles_x, ty = local / cam.tiles_x;
  const int64_t e0 = static_cast<int64_t>(i0) - t;  // slot of the tile's item 1
  for (int q = threadIdx.x; q < T * T; q += 256) {
    const int px = tx * T + q % T, py = ty * T + q / T;
    if (px >= cam.width || py >= cam.height) continue;
    const int64_t pix = cam.pix_base + static_cast<int64_t>(py) * cam.width + px;
    float4 s = reinterpret_cast<const float4*>(a.acc)[pix];
    float lg = OIT ? a.acclog[pix] : 0.f;
    for (uint32_t k = 1; k < nk; ++k) {
      const int64_t e = e0 + k - 1;
      if (e >= a.split_slots) break;
      const float4 x = a.split4[e * (T * T) + q];
      s.x += x.x;
      s.y += x.y;
      s.z += x.z;
      s.w += x.w;
      if (OIT) lg += a.splitlog[e * (T * T) + q];
    }
    if (OIT)
      write_pixel_oit(a, pix, s.x, s.y, s.z, s.w, __expf(lg));
    else
      write_pixel(a, pix, s.x, s.y, s.z, s.w);
  }
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

// Moments about the wave block's centre.  A lane sums, per pixel of its
// splat's walk, e = G dL/da against the pixel centre's offset xc from the
// block centre (a compile-time constant per column: no per-pixel dx or dx^2
// for the moments) and folds each row with dy = pixel y - splat y:
//   X1 = sum e xc, X2 = sum e xc^2, XY = sum e xc dy, My = sum e dy,
//   Myy = sum e dy^2, S = sum e.
// With dx = xc - m (m the splat centre's offset from the block centre) the
// moments about the splat centre follow once per splat:
//   Mx = X1 - m S,  Mxx = X2 - 2 m X1 + m^2 S,  Mxy = XY - m My,
// whose rounding is bounded like that of summing e dx directly (|xc| + |m|
// bounds |dx| over the block).
struct BlockMoments {
  float X1 = 0.f, X2 = 0.f, XY = 0.f, My = 0.f, Myy = 0.f, S = 0.f;
};

__device__ __forceinline__ void fold_row(BlockMoments& M, float dy, float S0, float S1, float S2) {
  M.S += S0;
  M.X1 += S1;
  M.X2 += S2;
  M.My = fmaf(dy, S0, M.My);
  M.XY = fmaf(dy, S1, M.XY);
  M.Myy = fmaf(dy * dy, S0, M.Myy);
}

__device__ __forceinline__ BlockMoments shfl_sum(BlockMoments M, int d) {
  M.X1 += __shfl_xor(M.X1, d, kWave);
  M.X2 += __shfl_xor(M.X2, d, kWave);
  M.XY += __shfl_xor(M.XY, d, kWave);
  M.My += __shfl_xor(M.My, d, kWave);
  M.Myy += __shfl_xor(M.Myy, d, kWave);
  M.S += __shfl_xor(M.S, d, kWave);
  return M;
}

// The five 2D-gradient sums from the block moments: the dq factors of the
// mean and conic gradients (dq = -a e / 2 per pixel, with a = amp G; the
// staged conic is scaled by log2(e) / 2, undone here).  `amp` multiplies the
// sums once (1 where the moments already carry the amplitude).
__device__ __forceinline__ void geom_sums(const BlockMoments& M, float m, float amp, float A, float B2, float Cc,
                                          float* o) {
  const float Mx = fmaf(-m, M.S, M.X1);
  const float Mxx = fmaf(m, fmaf(m, M.S, -2.f * M.X1), M.X2);
  const float Mxy = fmaf(-m, M.My, M.XY);
  const float ampc = amp * kTwoLn2;
  o[0] = ampc * (A * Mx + 0.5f * B2 * M.My);
  o[1] = ampc * (0.5f * B2 * Mx + Cc * M.My);
  o[2] = -0.5f * amp * Mxx;
  o[3] = -amp * Mxy;
  o[4] = -0.5f * amp * M.Myy;
}

// One chunk of the backward for one wave: up to 64 splats of the wave's
// culled list, one per lane, each walked over the wave's 8x8 pixel block.
// Per splat the lane sums, with G = exp(-q/2) and e = G dL/da, the block
// moments of e (three FMAs a pixel, see BlockMoments) and sum G gbar.  The
// splat's amplitude multiplies them once at the end.  The lane's nine
// partial 2D gradient sums are written to out[j][lane].  A lane past the
// end of the list gets a negative cutoff, so no pixel passes.
//
// All lanes walk the same pixel at the same time, so the per-pixel factors
// (gbar, s) are read from LDS at a wave-uniform address (a broadcast).
template <int T, bool CUT>
__device__ __forceinline__ void bwd_chunk(const TileCtx<T>& c, int c0, int m, const uint8_t* list,
                                          const StagedRec* s_rec, const float4* pd_wave,
                                          float (*out)[kWave], float tau) {
  const int j = c0 + c.lane;
  const bool valid = j < m;
  const int kr = valid ? list[j] : 0;
  const StagedRec r = s_rec[kr];
  const float amp = r.r1.y, cr = r.r1.z, cg = r.r1.w, cb = r.r2.x;
  BlockMoments M;
  float g_r = 0.f, g_g = 0.f, g_b = 0.f;
  const float A = r.r0.z, B2 = r.r0.w, Cc = r.r1.x;
  const float cut = valid ? (CUT ? r.r2.y : tau) : -1.f;
  // first pixel centre of the block relative to the tile's centre (exact),
  // so dx = (ex0 + col) - mx matches the forward's
  const float ex0 = static_cast<float>(c.bx0 - c.fx0) + 0.5f;
  const float ey0 = static_cast<float>(c.by0 - c.fy0) + 0.5f;
  float yrow = ey0;  // this row's pixel centre (exact: ey0 + row)
#pragma unroll 1
  for (int row = 0; row < 8; ++row, yrow += 1.f) {
    const float dy = yrow - r.r0.y;
    const float B2dy = B2 * dy, Cdy2 = (Cc * dy) * dy;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f;
#pragma unroll
    for (int col = 0; col < 8; ++col) {
      const float xc = static_cast<float>(col) - 3.5f;
      const float dx = (ex0 + static_cast<float>(col)) - r.r0.x;
      const float q = quad_form(A, B2dy, Cdy2, dx);
      const float4 pd = pd_wave[row * 8 + col];  // wave-uniform LDS address: a broadcast read
      const float Gq = q <= cut ? falloff(q) : 0.f;
      const float dLda = fmaf(pd.x, cr, fmaf(pd.y, cg, fmaf(pd.z, cb, -pd.w)));
      const float e = Gq * dLda;
      S0 += e;
      S1 = fmaf(e, xc, S1);
      S2 = fmaf(e, xc * xc, S2);
      g_r = fmaf(Gq, pd.x, g_r);
      g_g = fmaf(Gq, pd.y, g_g);
      g_b = fmaf(Gq, pd.z, g_b);
    }
    fold_row(M, dy, S0, S1, S2);
  }
  // dL/dc = amp sum G gbar, dL/damp = sum G dL/da
  const int l = c.lane;
  float o[5];
  geom_sums(M, r.r0.x - (ex0 + 3.5f), amp, A, B2, Cc, o);
#pragma unroll
  for (int q = 0; q < 5; ++q) out[q][l] = o[q];
  out[5][l] = amp * g_r;
  out[6][l] = amp * g_g;
  out[7][l] = amp * g_b;
  out[8][l] = M.S;
}

// A short chunk (at most 64 / K splats, K = 2, 4 or 8), which would leave
// most lanes of bwd_chunk idle: K lanes share a splat, lane group g walking
// rows [g 8/K, (g+1) 8/K) of the block, and the groups' sums are added with
// cross-lane shuffles in a fixed order.  The groups visit different pixels
// at the same time, so the per-pixel factors come from this wave's copy in
// LDS (s_pd, 64 entries) at per-group addresses.  The arithmetic per pixel
// is that of bwd_chunk.
template <int T, bool CUT, int K>
__device__ __forceinline__ void bwd_chunk_split(const TileCtx<T>& c, int c0, int m, const uint8_t* list,
                                                const StagedRec* s_rec, const float4* s_pd, float (*out)[kWave],
                                                float tau) {
  constexpr int S = kWave / K;  // splats per chunk
  constexpr int R = 8 / K;      // rows per lane group
  const int g = c.lane / S;
  const int slot = c.lane % S;
  const int j = c0 + slot;
  const bool valid = j < m;
  const int kr = valid ? list[j] : 0;
  const StagedRec r = s_rec[kr];
  const float amp = r.r1.y, cr = r.r1.z, cg = r.r1.w, cb = r.r2.x;
  BlockMoments M;
  float g_r = 0.f, g_g = 0.f, g_b = 0.f;
  const float A = r.r0.z, B2 = r.r0.w, Cc = r.r1.x;
  const float cut = valid ? (CUT ? r.r2.y : tau) : -1.f;
  const float ex0 = static_cast<float>(c.bx0 - c.fx0) + 0.5f;
  const float ey0 = static_cast<float>(c.by0 - c.fy0 + g * R) + 0.5f;  // first row of this group
  const float4* pd_rows = s_pd + g * R * 8;
#pragma unroll
  for (int row = 0; row < R; ++row) {
    const float dy = (ey0 + static_cast<float>(row)) - r.r0.y;
    const float B2dy = B2 * dy, Cdy2 = (Cc * dy) * dy;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f;
#pragma unroll
    for (int col = 0; col < 8; ++col) {
      const float xc = static_cast<float>(col) - 3.5f;
      const float dx = (ex0 + static_cast<float>(col)) - r.r0.x;
      const float q = quad_form(A, B2dy, Cdy2, dx);
      const float4 pd = pd_rows[row * 8 + col];
      const float Gq = q <= cut ? falloff(q) : 0.f;
      const float dLda = fmaf(pd.x, cr, fmaf(pd.y, cg, fmaf(pd.z, cb, -pd.w)));
      const float e = Gq * dLda;
      S0 += e;
      S1 = fmaf(e, xc, S1);
      S2 = fmaf(e, xc * xc, S2);
      g_r = fmaf(Gq, pd.x, g_r);
      g_g = fmaf(Gq, pd.y, g_g);
      g_b = fmaf(Gq, pd.z, g_b);
    }
    fold_row(M, dy, S0, S1, S2);
  }
#pragma unroll
  for (int d = S; d < kWave; d <<= 1) {
    M = shfl_sum(M, d);
    g_r += __shfl_xor(g_r, d, kWave);
    g_g += __shfl_xor(g_g, d, kWave);
    g_b += __shfl_xor(g_b, d, kWave);
  }
  if (g == 0) {
    float o[5];
    geom_sums(M, r.r0.x - (ex0 + 3.5f), amp, A, B2, Cc, o);
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q][slot] = o[q];
    out[5][slot] = amp * g_r;
    out[6][slot] = amp * g_g;
    out[7][slot] = amp * g_b;
    out[8][slot] = M.S;
  }
}

// The OIT chunk (Eq. 2): as bwd_chunk, plus the coverage term.  A layer's
// opacity alpha = u G (clamped to [0, 1], no gradient where clamped) gets
// dL/dalpha = -k / (1 - alpha) with k from pixel_factors, so per pixel
// dq = -G (amp dL/da + u dL/dalpha) / 2, and the tenth output is
// dL/du = sum G dL/dalpha.  The moments therefore carry the amplitude.
template <int T>
__device__ __forceinline__ void bwd_chunk_oit(const TileCtx<T>& c, int c0, int m, const uint8_t* list,
                                              const StagedRec* s_rec,
                                              const float4* pd_wave, const float* pk_wave,
                                              float (*out)[kWave], float tau) {
  const int j = c0 + c.lane;
  const bool valid = j < m;
  const int kr = valid ? list[j] : 0;
  const StagedRec r = s_rec[kr];
  const float u = r.r2.z;
  const float amp = r.r1.y, cr = r.r1.z, cg = r.r1.w, cb = r.r2.x;
  BlockMoments M;
  float g_r = 0.f, g_g = 0.f, g_b = 0.f, g_amp = 0.f, g_u = 0.f;
  const float A = r.r0.z, B2 = r.r0.w, Cc = r.r1.x;
  const float cut = valid ? tau : -1.f;
  const float ex0 = static_cast<float>(c.bx0 - c.fx0) + 0.5f;
  const float ey0 = static_cast<float>(c.by0 - c.fy0) + 0.5f;
  float yrow = ey0;  // this row's pixel centre (exact: ey0 + row)
#pragma unroll 1
  for (int row = 0; row < 8; ++row, yrow += 1.f) {
    const float dy = yrow - r.r0.y;
    const float B2dy = B2 * dy, Cdy2 = (Cc * dy) * dy;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f;
#pragma unroll
    for (int col = 0; col < 8; ++col) {
      const float xc = static_cast<float>(col) - 3.5f;
      const float dx = (ex0 + static_cast<float>(col)) - r.r0.x;
      const float q = quad_form(A, B2dy, Cdy2, dx);
      const float4 pd = pd_wave[row * 8 + col];  // wave-uniform LDS address: a broadcast read
      const float k = pk_wave[row * 8 + col];
      const float Gq = q <= cut ? falloff(q) : 0.f;
      const float dLda = fmaf(pd.x, cr, fmaf(pd.y, cg, fmaf(pd.z, cb, -pd.w)));
      const float al = u * Gq;
      // hardware reciprocal (within 1 ulp) instead of an IEEE division
      const float dLdal = (al > 0.f && al < 1.f) ? -k * __builtin_amdgcn_rcpf(1.f - al) : 0.f;
      const float e = Gq * fmaf(amp, dLda, u * dLdal);
      S0 += e;
      S1 = fmaf(e, xc, S1);
      S2 = fmaf(e, xc * xc, S2);
      g_r = fmaf(Gq, pd.x, g_r);
      g_g = fmaf(Gq, pd.y, g_g);
      g_b = fmaf(Gq, pd.z, g_b);
      g_amp = fmaf(Gq, dLda, g_amp);
      g_u = fmaf(Gq, dLdal, g_u);
    }
    fold_row(M, dy, S0, S1, S2);
  }
  const int l = c.lane;
  float o[5];
  geom_sums(M, r.r0.x - (ex0 + 3.5f), 1.f, A, B2, Cc, o);
#pragma unroll
  for (int q = 0; q < 5; ++q) out[q][l] = o[q];
  out[5][l] = amp * g_r;
  out[6][l] = amp * g_g;
  out[7][l] = amp * g_b;
  out[8][l] = g_amp;
  out[9][l] = g_u;
}

// bwd_chunk_oit for a short chunk, with K lanes per splat as in
// bwd_chunk_split (per-pixel factors and coverage factors from LDS).
template <int T, int K>
__device__ __forceinline__ void bwd_chunk_oit_split(const TileCtx<T>& c, int c0, int m, const uint8_t* list,
                                                    const StagedRec* s_rec, const float4* s_pd,
                                                    const float* s_pk, float (*out)[kWave], float tau) {
  constexpr int S = kWave / K;  // splats per chunk
  constexpr int R = 8 / K;      // rows per lane group
  const int g = c.lane / S;
  const int slot = c.lane % S;
  const int j = c0 + slot;
  const bool valid = j < m;
  const int kr = valid ? list[j] : 0;
  const StagedRec r = s_rec[kr];
  const float u = r.r2.z;
  const float amp = r.r1.y, cr = r.r1.z, cg = r.r1.w, cb = r.r2.x;
  BlockMoments M;
  float g_r = 0.f, g_g = 0.f, g_b = 0.f, g_amp = 0.f, g_u = 0.f;
  const float A = r.r0.z, B2 = r.r0.w, Cc = r.r1.x;
  const float cut = valid ? tau : -1.f;
  const float ex0 = static_cast<float>(c.bx0 - c.fx0) + 0.5f;
  const float ey0 = static_cast<float>(c.by0 - c.fy0 + g * R) + 0.5f;  // first row of this group
  const float4* pd_rows = s_pd + g * R * 8;
  const float* pk_rows = s_pk + g * R * 8;
#pragma unroll
  for (int row = 0; row < R; ++row) {
    const float dy = (ey0 + static_cast<float>(row)) - r.r0.y;
    const float B2dy = B2 * dy, Cdy2 = (Cc * dy) * dy;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f;
#pragma unroll
    for (int col = 0; col < 8; ++col) {
      const float xc = static_cast<float>(col) - 3.5f;
      const float dx = (ex0 + static_cast<float>(col)) - r.r0.x;
      const float q = quad_form(A, B2dy, Cdy2, dx);
      const float4 pd = pd_rows[row * 8 + col];
      const float k = pk_rows[row * 8 + col];
      const float Gq = q <= cut ? falloff(q) : 0.f;
      const float dLda = fmaf(pd.x, cr, fmaf(pd.y, cg, fmaf(pd.z, cb, -pd.w)));
      const float al = u * Gq;
      const float dLdal = (al > 0.f && al < 1.f) ? -k * __builtin_amdgcn_rcpf(1.f - al) : 0.f;
      const float e = Gq * fmaf(amp, dLda, u * dLdal);
      S0 += e;
      S1 = fmaf(e, xc, S1);
      S2 = fmaf(e, xc * xc, S2);
      g_r = fmaf(Gq, pd.x, g_r);
      g_g = fmaf(Gq, pd.y, g_g);
      g_b = fmaf(Gq, pd.z, g_b);
      g_amp = fmaf(Gq, dLda, g_amp);
      g_u = fmaf(Gq, dLdal, g_u);
    }
    fold_row(M, dy, S0, S1, S2);
  }
#pragma unroll
  for (int d = S; d < kWave; d <<= 1) {
    M = shfl_sum(M, d);
    g_r += __shfl_xor(g_r, d, kWave);
    g_g += __shfl_xor(g_g, d, kWave);
    g_b += __shfl_xor(g_b, d, kWave);
    g_amp += __shfl_xor(g_amp, d, kWave);
    g_u += __shfl_xor(g_u, d, kWave);
  }
  if (g == 0) {
    float o[5];
    geom_sums(M, r.r0.x - (ex0 + 3.5f), 1.f, A, B2, Cc, o);
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q][slot] = o[q];
    out[5][slot] = amp * g_r;
    out[6][slot] = amp * g_g;
    out[7][slot] = amp * g_b;
    out[8][slot] = g_amp;
    out[9][slot] = g_u;
  }
}

// The backward's per-pixel factors for pixel (px, py) of view `cam`:
// gbar = dL/dC / D and s = gbar . C (zero outside the image), and the pixel's
// share of the background gradients dL/dc_B (rgb) and dL/dw_B.
//
// OIT (Eq. 2, C = P c_B + (1 - P) N / D): gbar = dL/dC (1 - P) / D and
// s = gbar . (N / D), so that dL/da = gbar . c - s as for Eq. 7, and the
// coverage factor k = P dL/dC . (c_B - N / D), so that a layer's opacity
// alpha gets dL/dalpha = -k / (1 - alpha); dL/dc_B = P dL/dC, dL/dw_B = 0.
template <bool OIT>
__device__ __forceinline__ void pixel_factors(const RasterArgs& a, const DevCamera& cam, int px, int py,
                                              float4* pd_o, float* kcov_o, float* bacc) {
  const float wbg = a.globals[2];
  const float bgr = a.globals[3], bgg = a.globals[4], bgb = a.globals[5];
  float4 pd = make_float4(0.f, 0.f, 0.f, 0.f);
  float kcov = 0.f;
  bacc[0] = bacc[1] = bacc[2] = bacc[3] = 0.f;
  if (px < cam.width && py < cam.height) {
    const int64_t pix = cam.pix_base + static_cast<int64_t>(py) * cam.width + px;
    const float D = a.den[pix];
    const float g0 = a.dL_drgb[3 * pix], g1 = a.dL_drgb[3 * pix + 1], g2 = a.dL_drgb[3 * pix + 2];
    if (OIT) {
      const float4 o = a.oit[pix];  // (N / D, P)
      const float P = o.w;
      const float f = D != 0.f ? (1.f - P) / D : 0.f;
      pd.x = g0 * f;
      pd.y = g1 * f;
      pd.z = g2 * f;
      pd.w = pd.x * o.x + pd.y * o.y + pd.z * o.z;
      kcov = P * (g0 * (bgr - o.x) + g1 * (bgg - o.y) + g2 * (bgb - o.z));
      bacc[0] = g0 * P;
      bacc[1] = g1 * P;
      bacc[2] = g2 * P;
    } else if (D != 0.f) {
      const float iD = 1.f / D;
      pd.x = g0 * iD;
      pd.y = g1 * iD;
      pd.z = g2 * iD;
      pd.w = pd.x * a.rgb[3 * pix] + pd.y * a.rgb[3 * pix + 1] + pd.z * a.rgb[3 * pix + 2];
      bacc[0] = wbg * pd.x;
      bacc[1] = wbg * pd.y;
      bacc[2] = wbg * pd.z;
      bacc[3] = pd.x * bgr + pd.y * bgg + pd.z * bgb - pd.w;
    } else {
      // C is the background colour where the denominator vanishes
      bacc[0] = g0;
      bacc[1] = g1;
      bacc[2] = g2;
    }
  }
  *pd_o = pd;
  *kcov_o = kcov;
}

// Tile 16 asks the compiler for five resident waves per SIMD with Eq. 7 (at
// most 102 VGPRs): the short-chunk path would otherwise raise the register
// count and cost a wave.  With Eq. 2 it asks for four (at most 128 VGPRs, no
// spills; the unbounded kernel takes 165, three waves): five would fit the
// LDS but spill 19 registers, which measured slower.
template <int T, bool OIT>
constexpr int bwd_min_blocks() {
  return T == 16 ? (OIT ? 4 : 5) : 1;
}

// Backward: each thread first forms its pixel's factors (pixel_factors)
// into LDS; the tile's first work item also stores the tile's
// background-gradient partial sums.  Then the same staging and per-wave
// culling as the forward, but lanes own splats of the wave's culled list and
// walk the wave's pixel block (see bwd_chunk), so a splat's nine gradient
// sums stay in registers.  A chunk of at most 32 splats (the tail of a
// wave's list) shares each splat among 2, 4 or 8 lanes instead
// (bwd_chunk_split, bwd_chunk_oit_split).
//
// The waves of a tile merge their sums without atomics.  Thread k owns
// staged record k.  The waves process their chunks in lockstep rounds (one
// chunk each per round); after a round every wave's sums sit in LDS, and each
// owner adds the entries of its record -- found through the per-wave list
// positions recorded by the culling -- into registers, waves in a fixed
// order.  At the end of the batch the owner stores the record's sums, zeros
// included, with plain stores at the pair's Gaussian-major slot.  For given
// tile lists the summation order is fixed, so the result does not vary from
// run to run (the order in which a record's per-wave sums are added follows
// the rounds that reach them, i.e. the list positions).
template <int T, int S, bool CUT, bool OIT, bool PERSIST>
__global__ __launch_bounds__(TileGeom<T>::kThreads, (bwd_min_blocks<T, OIT>())) void raster_bwd_kernel(
    RasterArgs a) {
  using G = TileGeom<T>;
  constexpr int kB = S;  // records staged per batch (thread k < kB owns record k)
  static_assert(kB <= G::kThreads, "every staged record needs an owner thread");
  static_assert(kB <= 256, "the culled lists hold 8-bit record indices");
  constexpr int NV = OIT ? 10 : 9;  // sums per (tile, splat) pair
  __shared__ StagedRec s_rec[kB];
  __shared__ uint32_t s_slot[kB];
  __shared__ __align__(16) uint8_t s_list[G::kWaves * kB];
  __shared__ uint16_t s_pos[G::kWaves * kB];
  __shared__ float s_part[G::kWaves][NV][kWave];
  __shared__ int s_m[G::kWaves];
  __shared__ float4 s_pd[G::kThreads];            // per-pixel factors, thread order
  __shared__ float s_pk[OIT ? G::kThreads : 1];   // OIT: per-pixel coverage factors
  __shared__ float s_bg[G::kWaves][4];
  __shared__ uint32_t s_item;
  // the forward's culling masks, if it stored them for these lists with the
  // same early-out setting
  const uint64_t* masks_in =
      (a.masks && a.flags->cull_masks == (kCullMasks | (CUT ? 2u : 0u))) ? a.masks : nullptr;
  const uint32_t n_items = a.items[a.total_tiles];
  uint32_t item = PERSIST ? claim_item(a, &s_item) : blockIdx.x;
  while (item < n_items) {
    TileCtx<T> c;
    const DevCamera* cam;
    tile_setup<T>(a, item, c, cam);

    // every thread's per-pixel factors into LDS, where the chunks read them at
    // wave-uniform (broadcast) or per-lane addresses; the tile's first work
    // item also stores the tile's background-gradient partial sums
    {
      float4 pd;
      float kcov, bacc[4];
      pixel_factors<OIT>(a, *cam, c.px, c.py, &pd, &kcov, bacc);
      s_pd[threadIdx.x] = pd;
      if (OIT) s_pk[threadIdx.x] = kcov;
      if (c.k == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float sj = wave_sum(bacc[j]);
          if (c.lane == 0) s_bg[c.wave][j] = sj;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
          float sj = 0.f;
#pragma unroll
          for (int w = 0; w < G::kWaves; ++w) sj += s_bg[w][threadIdx.x];
          a.tilepart[c.tile * 4 + threadIdx.x] = sj;
        }
      }
    }
    const float4* pd_wave = s_pd + c.wave * kWave;
    const float* pk_wave = OIT ? s_pk + c.wave * kWave : nullptr;
    const float tau = a.tau;
    const int own = threadIdx.x;  // staged record owned by this thread (if < kB)
    for (uint32_t b = c.start; b < c.end; b += kB) {
      const int m = stage_and_cull<T, kB, true, CUT, OIT, false, uint8_t>(a, c, b, s_rec, s_slot, s_list, s_pos,
                                                                          nullptr, masks_in);
      const int cnt = static_cast<int>(min(static_cast<uint32_t>(kB), c.end - b));
      if (c.lane == 0) s_m[c.wave] = m;
      __syncthreads();
      int rounds = 0;
#pragma unroll
      for (int w = 0; w < G::kWaves; ++w) rounds = max(rounds, (s_m[w] + kWave - 1) / kWave);
      const uint8_t* list = s_list + c.wave * kB;
      float acc[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) acc[q] = 0.f;
      for (int r = 0; r < rounds; ++r) {
        const int left = m - r * kWave;  // splats in this wave's chunk of the round
        if (left > 0) {
          const float4* pdl = pd_wave;
          if (OIT) {
            const float* pkl = pk_wave;
            if (left > kWave / 2)
              bwd_chunk_oit<T>(c, r * kWave, m, list, s_rec, pd_wave, pk_wave, s_part[c.wave], tau);
            else if (left > kWave / 4)
              bwd_chunk_oit_split<T, 2>(c, r * kWave, m, list, s_rec, pdl, pkl, s_part[c.wave], tau);
            else if (left > kWave / 8)
              bwd_chunk_oit_split<T, 4>(c, r * kWave, m, list, s_rec, pdl, pkl, s_part[c.wave], tau);
            else
              bwd_chunk_oit_split<T, 8>(c, r * kWave, m, list, s_rec, pdl, pkl, s_part[c.wave], tau);
          } else {
            if (left > kWave / 2)
              bwd_chunk<T, CUT>(c, r * kWave, m, list, s_rec, pd_wave, s_part[c.wave], tau);
            else if (left > kWave / 4)
              bwd_chunk_split<T, CUT, 2>(c, r * kWave, m, list, s_rec, pdl, s_part[c.wave], tau);
            else if (left > kWave / 8)
              bwd_chunk_split<T, CUT, 4>(c, r * kWave, m, list, s_rec, pdl, s_part[c.wave], tau);
            else
              bwd_chunk_split<T, CUT, 8>(c, r * kWave, m, list, s_rec, pdl, s_part[c.wave], tau);
          }
        }
        __syncthreads();
        if (own < cnt) {
#pragma unroll
          for (int w = 0; w < G::kWaves; ++w) {
            const int p = s_pos[w * kB + own];  // 0xffff: culled by wave w
            if ((p >> 6) == r) {
#pragma unroll
              for (int q = 0; q < NV; ++q) acc[q] += s_part[w][q][p & (kWave - 1)];
            }
          }
        }
        __syncthreads();
      }
      if (own < cnt) {
        const uint32_t sl = s_slot[own];
        if (sl < a.capacity) {
          float3* dst = a.part + 3 * static_cast<int64_t>(sl);
          dst[0] = make_float3(acc[0], acc[1], acc[2]);
          dst[1] = make_float3(acc[3], acc[4], acc[5]);
          dst[2] = make_float3(acc[6], acc[7], acc[8]);
          if (OIT) a.du[sl] = acc[NV - 1];
        }
      }
    }
    if (!PERSIST) break;
    item = claim_item(a, &s_item);  // (its first barrier: the shared arrays are free again)
  }
}

// ---- Sorted alpha blending (Eq. 6): the baseline the method removes the
// sort from.  The splats are those of the weighted sum (projected with the
// DIR weight, so a record's amplitude is the opacity u), ordered per tile by
// camera depth and composited front to back.

// One workgroup per tile: the tile's list, keyed by (depth bits, list
// position), is sorted in LDS by a bitonic network over the next power of two
// (padding keys sort last), and the entries (id and Gaussian-major slot) are
// then moved to their sorted positions: every thread first reads the entries
// its positions receive, then, after a barrier, writes them.  Binning leaves
// every list in increasing id order, so ties in depth stay in id order.  An
// instance holds CAP keys and sorts the lists of length lo < l <= CAP; the
// largest instance raises a flag for lists longer than kSortMax, which stay
// unsorted.  Three instances (16, 64 and 128 KB of LDS): most lists are
// short, and the smaller instances let more workgroups share a CU.
constexpr int kSortSmall = 2048;
constexpr int kSortMid = 8192;

template <int CAP>
__global__ __launch_bounds__(1024) void sort_tiles_kernel(const DevCamera* cams, int32_t nv, const DevSplat* rec,
                                                          int64_t n, const uint32_t* tile_start, uint2* ent,
                                                          int64_t capacity, int lo, DevFlags* flags) {
  constexpr int R = CAP / 1024;  // list positions per thread
  __shared__ uint64_t keys[CAP];
  const int tile = static_cast<int>(blockIdx.x);
  // entries move: culling masks stored for the old positions no longer apply
  if (CAP == kSortSmall && tile == 0 && threadIdx.x == 0) flags->cull_masks = 0u;
  const uint64_t cap = static_cast<uint64_t>(capacity);
  uint64_t s = tile_start[tile], e = tile_start[tile + 1];
  s = s < cap ? s : cap;
  e = e < cap ? e : cap;
  if (e <= s + 1 || e - s <= static_cast<uint64_t>(lo)) return;
  if (e - s > static_cast<uint64_t>(CAP)) {
    if (CAP == kSortMax && threadIdx.x == 0) flags->sort_overflow = 1u;
    return;
  }
  const int len = static_cast<int>(e - s);
  const int v = find_view(cams, nv, tile);
  int npow = 2;
  while (npow < len) npow <<= 1;
  for (int k = threadIdx.x; k < npow; k += 1024) {
    uint64_t key = ~0ull;
    if (k < len) {
      const uint32_t id = ent[s + k].x;
      const uint32_t depth = rec[static_cast<int64_t>(v) * n + id].slot.w;
      key = (static_cast<uint64_t>(depth) << 32) | static_cast<uint32_t>(k);
    }
    keys[k] = key;
  }
  __syncthreads();
  for (int size = 2; size <= npow; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (npow >> 1); i += 1024) {
        const int a = (i / stride) * 2 * stride + (i % stride);
        const int b = a + stride;
        const bool up = (a & size) == 0;
        const uint64_t x = keys[a], y = keys[b];
        if ((x > y) == up) {
          keys[a] = y;
          keys[b] = x;
        }
      }
      __syncthreads();
    }
  }
  uint2 moved[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = threadIdx.x + r * 1024;
    if (k < len) moved[r] = ent[s + static_cast<uint32_t>(keys[k])];
  }
  __syncthreads();  // every old entry has been read
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = threadIdx.x + r * 1024;
    if (k < len) ent[s + k] = moved[r];
  }
}

// One workgroup per tile (no splitting: the composition is sequential), the
// same staging and per-wave culling as the weighted sum (the culled list
// keeps the depth order); per pixel alpha = min(alpha_max, u G), layers
// below alpha_min skipped, C += c alpha T and T *= 1 - alpha, a pixel stops
// once T < t_min and the tile once all its pixels have stopped.
template <int T>
__global__ __launch_bounds__(TileGeom<T>::kThreads) void raster_sorted_kernel(RasterArgs a, float alpha_max,
                                                                              float alpha_min, float t_min,
                                                                              float* out_T) {
  using G = TileGeom<T>;
  __shared__ StagedRec s_rec[G::kBatch];
  __shared__ __align__(16) uint8_t s_list[G::kWaves * G::kBatch];
  TileCtx<T> c;
  const int tile = static_cast<int>(blockIdx.x);
  c.v = find_view(a.cams, a.nv, tile);
  const DevCamera* cam = &a.cams[c.v];
  const int local = tile - cam->tile_base;
  c.tile = tile;
  c.tx = local % cam->tiles_x;
  c.ty = local / cam->tiles_x;
  c.n = a.n;
  const uint64_t cap = static_cast<uint64_t>(a.capacity);
  uint64_t s = a.tile_start[tile], e = a.tile_start[tile + 1];
  s = s < cap ? s : cap;
  e = e < cap ? e : cap;
  if (e < s) e = s;
  c.start = static_cast<uint32_t>(s);
  c.end = static_cast<uint32_t>(e);
  c.k = 0;
  c.nk = 1;
  c.wave = threadIdx.x / kWave;
  c.lane = threadIdx.x % kWave;
  c.bx0 = c.tx * T + (c.wave % (T / 8)) * G::kSub;
  c.by0 = c.ty * T + (c.wave / (T / 8)) * G::kSub;
  c.fx0 = c.tx * T + T / 2;
  c.fy0 = c.ty * T + T / 2;
  c.px = c.bx0 + (c.lane & 7);
  c.py = c.by0 + (c.lane >> 3);
  const bool inside = c.px < cam->width && c.py < cam->height;
  bool live = inside;
  float cr = 0.f, cg = 0.f, cb = 0.f, Tr = 1.f;
  const float pcx = static_cast<float>(c.px - c.fx0) + 0.5f;  // relative to the tile's centre
  const float pcy = static_cast<float>(c.py - c.fy0) + 0.5f;
  const float tau = a.tau;
  for (uint32_t b = c.start; b < c.end; b += G::kBatch) {
    const int m = stage_and_cull<T, G::kBatch, false, false, false, false, uint8_t>(a, c, b, s_rec, nullptr, s_list,
                                                                            nullptr);
    const uint8_t* list = s_list + c.wave * G::kBatch;
    for (int i = 0; i < m && live; ++i) {
      const StagedRec r = s_rec[list[i]];
      const float q = pair_q(r, pcx, pcy);
      const float al = fminf(alpha_max, r.r1.y * falloff(q));
      if (q <= tau && al >= alpha_min) {
        const float w = al * Tr;
        cr = fmaf(w, r.r1.z, cr);
        cg = fmaf(w, r.r1.w, cg);
        cb = fmaf(w, r.r2.x, cb);
        Tr *= 1.f - al;
        if (Tr < t_min) live = false;
      }
    }
    if (!__syncthreads_or(live ? 1 : 0)) break;
  }
  if (!inside) return;
  const int64_t pix = cam->pix_base + static_cast<int64_t>(c.py) * cam->width + c.px;
  a.out_rgb[3 * pix] = fmaf(Tr, a.globals[3], cr);
  a.out_rgb[3 * pix + 1] = fmaf(Tr, a.globals[4], cg);
  a.out_rgb[3 * pix + 2] = fmaf(Tr, a.globals[5], cb);
  out_T[pix] = Tr;
}

RasterArgs make_args(const Layout& L, void* ws, const void* pairs, int64_t capacity,
                     const wsr_params* P, const float* globals) {
  RasterArgs a = {};
  const PairView pv = pair_view(pairs, capacity);
  a.cams = at<DevCamera>(ws, L.off_cams);
  a.rec = at<DevSplat>(ws, L.off_rec);
  a.tile_start = at<uint32_t>(ws, L.off_tstart);
  a.ent = pv.ent;
  a.part = pv.part;
  a.n = L.n;
  a.capacity = capacity;
  a.nv = L.nv;
  a.tau = P->tau * kHalfLog2e;  // in the scale of the staged conic
  a.unnormalised = (P->flags & WSR_FLAG_UNNORMALISED) ? 1 : 0;
  a.globals = globals;
  a.items = at<uint32_t>(ws, L.off_items);
  a.tile_order = at<uint32_t>(ws, L.off_torder);
  a.total_tiles = L.total_tiles;
  a.acc = at<float>(ws, L.off_acc);
  // The forward's split-tile slots live in the pair buffer's partial-gradient
  // region, which the raster backward fills only later.  A tile of l pairs
  // has ceil(l / kItemSplats) - 1 items beyond its first, so at most
  // (capacity - 1) / kItemSplats slots exist; their T^2 x 20 bytes each fit
  // in the region's 36 bytes per pair for every tile size (T <= 32).
  a.split_slots = capacity > 0 ? (capacity - 1) / kItemSplats : 0;
  a.split4 = reinterpret_cast<float4*>(pv.part);
  a.splitlog = reinterpret_cast<float*>(a.split4 + a.split_slots * L.tile * L.tile);
  a.oit = at<float4>(ws, L.off_oit);
  a.acclog = at<float>(ws, L.off_acclog);
  a.du = pv.du;
  a.flags = at<DevFlags>(ws, L.off_flags);
  // The culling masks have 4 bytes per pair of the pair buffer; a capacity
  // too small for the per-tile rounding of the groups leaves them off.
  {
    const int64_t waves = static_cast<int64_t>(L.tile / 8) * (L.tile / 8);
    const int64_t words = (((capacity + 63) >> 6) + L.total_tiles + 2) * waves;
    a.masks = capacity > 0 && 8 * words <= 4 * capacity ? pv.masks : nullptr;
  }
  return a;
}

// Workgroups of `kernel` (with `threads` threads) the current device holds
// at once: its compute units times the workgroups one of them can host.
// Looked up once per kernel and device; 0 if the runtime cannot tell.
int64_t resident_workgroups(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int64_t> known;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(kernel, dev);
  const auto it = known.find(key);
  if (it != known.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int64_t r = static_cast<int64_t>(per_cu) * cus;
  known[key] = r;
  return r;
}

// Launch a raster kernel over the work items: one workgroup per item (the
// grid covers the upper bound of the item count; workgroups beyond the
// actual count exit at once), or, with a queue, the persistent kernel on as
// many workgroups as the device holds at once, claiming items from the
// queue (cleared here first) until none is left.
hipError_t launch_items(void (*grid_kernel)(RasterArgs), void (*persistent_kernel)(RasterArgs), RasterArgs a,
                        int64_t max_items, uint32_t* queue, int threads, hipStream_t st) {
  if (queue) {
    const int64_t r = resident_workgroups(reinterpret_cast<const void*>(persistent_kernel), threads);
    if (r > 0 && r < max_items) {
      a.queue = queue;
      const hipError_t e = launch_fill_zero(queue, sizeof(uint32_t), st);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(persistent_kernel, dim3(static_cast<unsigned>(r)), dim3(threads), 0, st, a);
      return hipGetLastError();
    }
  }
  a.queue = nullptr;
  hipLaunchKernelGGL(grid_kernel, dim3(static_cast<unsigned>(max_items)), dim3(threads), 0, st, a);
  return hipGetLastError();
}

template <int T, int S, bool COUNT, bool CUT, bool OIT>
hipError_t fwd_k(const RasterArgs& a, int64_t grid, uint32_t* queue, hipStream_t st) {
  return launch_items(raster_fwd_kernel<T, S, COUNT, CUT, OIT, false>, raster_fwd_kernel<T, S, COUNT, CUT, OIT, true>,
                      a, grid, queue, TileGeom<T>::kThreads, st);
}

template <int T, int S>
hipError_t fwd_ts(const RasterArgs& a, int64_t grid, bool count, bool cut, bool oit, uint32_t* queue,
                  hipStream_t st) {
  if (oit) return count ? fwd_k<T, S, true, false, true>(a, grid, queue, st) : fwd_k<T, S, false, false, true>(a, grid, queue, st);
  if (cut) return count ? fwd_k<T, S, true, true, false>(a, grid, queue, st) : fwd_k<T, S, false, true, false>(a, grid, queue, st);
  return count ? fwd_k<T, S, true, false, false>(a, grid, queue, st) : fwd_k<T, S, false, false, false>(a, grid, queue, st);
}

template <int T, int S, bool CUT, bool OIT>
hipError_t bwd_k(const RasterArgs& a, int64_t grid, uint32_t* queue, hipStream_t st) {
  return launch_items(raster_bwd_kernel<T, S, CUT, OIT, false>, raster_bwd_kernel<T, S, CUT, OIT, true>, a, grid,
                      queue, TileGeom<T>::kThreads, st);
}

template <int T, int S>
hipError_t bwd_ts(const RasterArgs& a, int64_t grid, bool cut, bool oit, uint32_t* queue, hipStream_t st) {
  if (oit) return bwd_k<T, S, false, true>(a, grid, queue, st);
  if (cut) return bwd_k<T, S, true, false>(a, grid, queue, st);
  return bwd_k<T, S, false, false>(a, grid, queue, st);
}

// Records staged per batch: tile 8 (one wave, 64 threads) stages 64; tiles
// 16 and 32 take 64 (tile 16 only), 128 or 256 (the default).
template <int T>
hipError_t fwd_t(const RasterArgs& a, int64_t grid, int64_t tiles, int batch, bool count, bool cut, bool oit,
                 uint32_t* queue, hipStream_t st) {
  hipError_t e;
  if constexpr (T == 8) {
    e = fwd_ts<8, 64>(a, grid, count, cut, oit, queue, st);
  } else {
    if (batch == 128)
      e = fwd_ts<T, 128>(a, grid, count, cut, oit, queue, st);
    else if (T == 16 && batch == 64)
      e = fwd_ts<16, 64>(a, grid, count, cut, oit, queue, st);
    else
      e = fwd_ts<T, 256>(a, grid, count, cut, oit, queue, st);
  }
  if (e != hipSuccess) return e;
  if (oit)
    raster_fwd_finalize<T, true><<<dim3(static_cast<unsigned>(tiles)), 256, 0, st>>>(a);
  else
    raster_fwd_finalize<T, false><<<dim3(static_cast<unsigned>(tiles)), 256, 0, st>>>(a);
  return hipGetLastError();
}

template <int T>
hipError_t bwd_t(const RasterArgs& a, int64_t grid, int batch, bool cut, bool oit, uint32_t* queue, hipStream_t st) {
  if constexpr (T == 8) {
    return bwd_ts<8, 64>(a, grid, cut, oit, queue, st);
  } else {
    if (batch == 128) return bwd_ts<T, 128>(a, grid, cut, oit, queue, st);
    if (T == 16 && batch == 64) return bwd_ts<16, 64>(a, grid, cut, oit, queue, st);
    return bwd_ts<T, 256>(a, grid, cut, oit, queue, st);
  }
}

}  // namespace

hipError_t launch_raster_fwd(const Layout& L, void* ws, const void* pairs, int64_t capacity,
                             const wsr_params* P, const float* globals, float* out_rgb,
                             float* out_den, int32_t* out_count, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  RasterArgs a = make_args(L, ws, pairs, capacity, P, globals);
  a.out_rgb = out_rgb;
  a.out_den = out_den;
  a.out_count = out_count;
  const bool cnt = out_count != nullptr;
  if (cnt) {
    const hipError_t e = launch_fill_zero(out_count, sizeof(int32_t) * L.total_pixels, st);
    if (e != hipSuccess) return e;
  }
  const int64_t grid = max_raster_items(L, capacity);
  const bool oit = (P->flags & WSR_FLAG_OIT) != 0;
  uint32_t* queue = (P->flags & WSR_FLAG_PERSISTENT) ? at<uint32_t>(ws, L.off_queue) : nullptr;
  const bool cut = P->alpha_cut > 0.f;
  switch (L.tile) {
    case 8: return fwd_t<8>(a, grid, L.total_tiles, P->batch, cnt, cut, oit, queue, st);
    case 32: return fwd_t<32>(a, grid, L.total_tiles, P->batch, cnt, cut, oit, queue, st);
    default: return fwd_t<16>(a, grid, L.total_tiles, P->batch, cnt, cut, oit, queue, st);
  }
}

hipError_t launch_raster_bwd(const Layout& L, void* ws, void* pairs, int64_t capacity,
                             const wsr_params* P, const float* globals, const float* dL_drgb,
                             const float* rgb, const float* den, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  RasterArgs a = make_args(L, ws, pairs, capacity, P, globals);
  a.dL_drgb = dL_drgb;
  a.rgb = rgb;
  a.den = den;
  a.tilepart = at<float>(ws, L.off_tilepart);
  const int64_t grid = max_raster_items(L, capacity);
  const bool oit = (P->flags & WSR_FLAG_OIT) != 0;
  uint32_t* queue = (P->flags & WSR_FLAG_PERSISTENT) ? at<uint32_t>(ws, L.off_queue) + 1 : nullptr;
  const bool cut = P->alpha_cut > 0.f;
  switch (L.tile) {
    case 8: return bwd_t<8>(a, grid, P->batch, cut, oit, queue, st);
    case 32: return bwd_t<32>(a, grid, P->batch, cut, oit, queue, st);
    default: return bwd_t<16>(a, grid, P->batch, cut, oit, queue, st);
  }
}

}  // namespace wsr

namespace wsr {

hipError_t launch_sort_tiles(const Layout& L, void* ws, void* pairs, int64_t capacity, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  const PairView pv = pair_view(pairs, capacity);
  const dim3 grid(static_cast<unsigned>(L.total_tiles));
  // the three instances sort disjoint sets of tiles
  const DevCamera* cams = at<DevCamera>(ws, L.off_cams);
  const DevSplat* rec = at<DevSplat>(ws, L.off_rec);
  const uint32_t* tstart = at<uint32_t>(ws, L.off_tstart);
  DevFlags* flags = at<DevFlags>(ws, L.off_flags);
  sort_tiles_kernel<kSortSmall><<<grid, 1024, 0, st>>>(cams, L.nv, rec, L.n, tstart, pv.ent, capacity, 0, flags);
  sort_tiles_kernel<kSortMid><<<grid, 1024, 0, st>>>(cams, L.nv, rec, L.n, tstart, pv.ent, capacity, kSortSmall, flags);
  sort_tiles_kernel<kSortMax><<<grid, 1024, 0, st>>>(cams, L.nv, rec, L.n, tstart, pv.ent, capacity, kSortMid, flags);
  return hipGetLastError();
}

hipError_t launch_raster_sorted(const Layout& L, void* ws, const void* pairs, int64_t capacity,
                                const wsr_params* P, const float* globals, float alpha_max, float alpha_min,
                                float t_min, float* out_rgb, float* out_T, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  RasterArgs a = make_args(L, ws, pairs, capacity, P, globals);
  a.masks = nullptr;  // the sorted lists are culled on their own
  a.out_rgb = out_rgb;
  const dim3 grid(static_cast<unsigned>(L.total_tiles));
  switch (L.tile) {
    case 8:
      raster_sorted_kernel<8><<<grid, TileGeom<8>::kThreads, 0, st>>>(a, alpha_max, alpha_min, t_min, out_T);
      break;
    case 32:
      raster_sorted_kernel<32><<<grid, TileGeom<32>::kThreads, 0, st>>>(a, alpha_max, alpha_min, t_min, out_T);
      break;
    default:
      raster_sorted_kernel<16><<<grid, TileGeom<16>::kThreads, 0, st>>>(a, alpha_max, alpha_min, t_min, out_T);
  }
  return hipGetLastError();
}

}  // namespace wsr
