// The training step around the renderer (Sec. 5, implementation details):
// the rendering loss of 3D Gaussian Splatting -- an l1 term plus a D-SSIM
// term weighted lambda = 0.2 -- with its gradient with respect to the
// rendered image, and the Adam update of the parameters.
//
//   L_v = (1 - lambda) mean|x - y| + lambda (1 - mean SSIM(x, y)),  L = mean_v L_v
//
// SSIM per colour channel (Wang et al. 2004): local statistics under an
// 11 x 11 Gaussian window (sigma 1.5) with zero padding, C1 = 0.01^2,
// C2 = 0.03^2.  The map depends on x through u = G*x, Sxx = G*x^2 and
// Sxy = G*(x y); the gradient of its mean is therefore
//   dmean/dx = (G*dS/du + 2 x G*dS/dSxx + y G*dS/dSxy) / P
// (the window is symmetric, so its adjoint is the same zero-padded filter).
//
// Two passes over 16 x 16 pixel tiles with a 5-pixel halo staged in LDS and
// the separable filter applied along rows, then columns:
//   loss_pass1: the five windowed statistics -> map, the three derivative
//               maps (to the workspace) and the tile's share of the loss;
//   loss_pass2: the three derivative maps filtered again -> dL/dx.
// The tile shares are summed in FP64 in a fixed order (loss_finalize).
#include <cmath>
#include <type_traits>
#include <mutex>

#include "adam.h"
#include "wsr_internal.h"

// Workspace of the allocation-free loss entry point: the derivative maps and
// per-tile shares of wsr_loss, in a device array of fixed size.  Every device
// the library runs on holds its own copy until the process ends.  In host
// code this name stands for a host-side shadow, not a device address: host
// code uses only the address hipGetSymbolAddress returns for the current
// device (loss_static_workspace).
static __device__ __align__(256) unsigned char scratch[WSR_LOSS_STATIC_BYTES];

namespace wsr {
namespace {

constexpr int kLT = 16;               // output tile edge
constexpr int kHalo = 5;              // window radius
constexpr int kLE = kLT + 2 * kHalo;  // staged edge (26)
constexpr int kLossViewsPerLaunch = 16;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

// Views of one launch, passed by value: sizes, first pixel of each view in
// the concatenated images, first 16x16 loss tile of each view (global over
// all views) and the loss scale 1 / (P_v V) of each view.
struct LossViews {
  int32_t nv;
  int32_t tile0;  // first tile of this launch (global index)
  int32_t width[kLossViewsPerLaunch];
  int32_t height[kLossViewsPerLaunch];
  int32_t tiles_x[kLossViewsPerLaunch];
  int32_t tile_base[kLossViewsPerLaunch + 1];  // local to the launch
  int64_t pix_base[kLossViewsPerLaunch];
  float scale[kLossViewsPerLaunch];
  float gauss[11];  // normalised window taps
};

struct LossArgs {
  const float* img;
  const float* target;
  float* dmaps;           // [3][channel][pixel] derivative maps
  double* part;           // [tile * 3 + channel] loss shares
  float* dL;
  int64_t total_pixels;
  float lambda;
};

struct TileWhere {
  int v, tx0, ty0;
};

__device__ __forceinline__ TileWhere loss_tile(const LossViews& lv, int t) {
  int v = 0;
  while (v + 1 < lv.nv && lv.tile_base[v + 1] <= t) ++v;
  const int local = t - lv.tile_base[v];
  return {v, (local % lv.tiles_x[v]) * kLT, (local / lv.tiles_x[v]) * kLT};
}

// Stage the (26 x 26) region of the tile in M sources -- channel `ch` of the
// interleaved [pix][3] images (stride 3) or planar maps (stride 1) -- with
// zeros outside the view, interleaved in LDS (source q in component q of a
// float2 or float4), so that a filter tap reads all of them at once.  Every
// load of the thread is issued before the first LDS store, so a workgroup
// pays one memory round trip for all M.
constexpr int kStageIters = (kLE * kLE + 255) / 256;

template <int M>
using StageVec = typename std::conditional<M == 2, float2, float4>::type;

template <int M>
__device__ __forceinline__ void stage(StageVec<M> (*dst)[kLE + 1], const float* const src[M], int stride, int ch,
                                      const LossViews& lv, const TileWhere& w) {
  static_assert(M == 2 || M == 3, "two or three interleaved sources");
  const int width = lv.width[w.v], height = lv.height[w.v];
  const int64_t base = lv.pix_base[w.v];
  float val[M][kStageIters];
#pragma unroll
  for (int it = 0; it < kStageIters; ++it) {
    const int k = threadIdx.x + 256 * it;
    const int r = k / kLE, cc = k % kLE;
    const int py = w.ty0 - kHalo + r, px = w.tx0 - kHalo + cc;
    const bool in = k < kLE * kLE && px >= 0 && py >= 0 && px < width && py < height;
    // outside the view the load reads the view's first pixel and is discarded
    const int64_t pix = base + (in ? static_cast<int64_t>(py) * width + px : 0);
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const float x = src[q][pix * stride + ch];
      val[q][it] = in ? x : 0.f;
    }
  }
#pragma unroll
  for (int it = 0; it < kStageIters; ++it) {
    const int k = threadIdx.x + 256 * it;
    if (k < kLE * kLE) {
      if constexpr (M == 2)
        dst[k / kLE][k % kLE] = make_float2(val[0][it], val[1][it]);
      else
        dst[k / kLE][k % kLE] = make_float4(val[0][it], val[1][it], val[2][it], 0.f);
    }
  }
}

__device__ __forceinline__ double block_sum_256(double x, double* sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = x;
  __syncthreads();
  const double t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void loss_pass1(LossArgs a, LossViews lv) {
  __shared__ float2 s_xy[kLE][kLE + 1];   // (x, y)
  __shared__ float4 s_h4[kLE][kLT + 1];   // row-filtered x, y, x^2, y^2
  __shared__ float s_h1[kLE][kLT + 1];    // row-filtered x y
  __shared__ double s_red[4];
  const int t = blockIdx.x, ch = blockIdx.y;
  const TileWhere w = loss_tile(lv, t);
  {
    const float* const src[2] = {a.img, a.target};
    stage<2>(s_xy, src, 3, ch, lv, w);
  }
  __syncthreads();
  // row pass of the separable filter: the 26 rows, the 16 output columns
  for (int k = threadIdx.x; k < kLE * kLT; k += 256) {
    const int r = k / kLT, c = k % kLT;
    float hx = 0.f, hy = 0.f, hxx = 0.f, hyy = 0.f, hxy = 0.f;
#pragma unroll
    for (int b = 0; b < 11; ++b) {
      const float gb = lv.gauss[b];
      const float2 xy = s_xy[r][c + b];
      const float x = xy.x, y = xy.y;
      hx = fmaf(gb, x, hx);
      hy = fmaf(gb, y, hy);
      hxx = fmaf(gb, x * x, hxx);
      hyy = fmaf(gb, y * y, hyy);
      hxy = fmaf(gb, x * y, hxy);
    }
    s_h4[r][c] = make_float4(hx, hy, hxx, hyy);
    s_h1[r][c] = hxy;
  }
  __syncthreads();
  const int i = threadIdx.x / kLT, j = threadIdx.x % kLT;
  const int px = w.tx0 + j, py = w.ty0 + i;
  double share = 0.0;
  if (px < lv.width[w.v] && py < lv.height[w.v]) {
    // column pass
    float u = 0.f, v = 0.f, sxx = 0.f, syy = 0.f, sxy = 0.f;
#pragma unroll
    for (int q = 0; q < 11; ++q) {
      const float gq = lv.gauss[q];
      const float4 h = s_h4[i + q][j];
      const float h1 = s_h1[i + q][j];
      u = fmaf(gq, h.x, u);
      v = fmaf(gq, h.y, v);
      sxx = fmaf(gq, h.z, sxx);
      syy = fmaf(gq, h.w, syy);
      sxy = fmaf(gq, h1, sxy);
    }
    const float a1 = 2.f * u * v + kC1;
    const float a2 = 2.f * (sxy - u * v) + kC2;
    const float b1 = u * u + v * v + kC1;
    const float b2 = (sxx - u * u) + (syy - v * v) + kC2;
    const float ib = 1.f / (b1 * b2);
    const float s = a1 * a2 * ib;
    const float d_u = (2.f * v * a2 - 2.f * v * a1) * ib - s * (2.f * u / b1 - 2.f * u / b2);
    const float d_sxx = -s / b2;
    const float d_sxy = 2.f * a1 * ib;
    const int64_t pix = lv.pix_base[w.v] + static_cast<int64_t>(py) * lv.width[w.v] + px;
    const int64_t P = a.total_pixels;
    a.dmaps[(0 * 3 + ch) * P + pix] = d_u;
    a.dmaps[(1 * 3 + ch) * P + pix] = d_sxx;
    a.dmaps[(2 * 3 + ch) * P + pix] = d_sxy;
    const float x = s_xy[i + kHalo][j + kHalo].x, y = s_xy[i + kHalo][j + kHalo].y;
    // this entry's part of L_v * V * P_v: (1 - lambda)|x - y| + lambda (1 - S)
    share = (1.0 - a.lambda) * fabs(static_cast<double>(x) - y) + a.lambda * (1.0 - static_cast<double>(s));
  }
  share = block_sum_256(share, s_red);
  if (threadIdx.x == 0) a.part[static_cast<int64_t>(lv.tile0 + t) * 3 + ch] = share * lv.scale[w.v];
}

__global__ __launch_bounds__(256) void loss_pass2(LossArgs a, LossViews lv) {
  __shared__ float4 s_m[kLE][kLE + 1];   // the three derivative maps (fourth component unused)
  __shared__ float4 s_h[kLE][kLT + 1];   // the same, row-filtered
  const int t = blockIdx.x, ch = blockIdx.y;
  const TileWhere w = loss_tile(lv, t);
  const int i = threadIdx.x / kLT, j = threadIdx.x % kLT;
  const int64_t P = a.total_pixels;
  {
    const float* const src[3] = {a.dmaps + (0 * 3 + ch) * P, a.dmaps + (1 * 3 + ch) * P, a.dmaps + (2 * 3 + ch) * P};
    stage<3>(s_m, src, 1, 0, lv, w);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kLE * kLT; k += 256) {
    const int r = k / kLT, c = k % kLT;
    float h0 = 0.f, h1 = 0.f, h2 = 0.f;
#pragma unroll
    for (int b = 0; b < 11; ++b) {
      const float gb = lv.gauss[b];
      const float4 m = s_m[r][c + b];
      h0 = fmaf(gb, m.x, h0);
      h1 = fmaf(gb, m.y, h1);
      h2 = fmaf(gb, m.z, h2);
    }
    s_h[r][c] = make_float4(h0, h1, h2, 0.f);
  }
  __syncthreads();
  float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 11; ++q) {
    const float gq = lv.gauss[q];
    const float4 h = s_h[i + q][j];
    f[0] = fmaf(gq, h.x, f[0]);
    f[1] = fmaf(gq, h.y, f[1]);
    f[2] = fmaf(gq, h.z, f[2]);
  }
  const int px = w.tx0 + j, py = w.ty0 + i;
  if (px >= lv.width[w.v] || py >= lv.height[w.v]) return;
  const int64_t pix = lv.pix_base[w.v] + static_cast<int64_t>(py) * lv.width[w.v] + px;
  const float x = a.img[3 * pix + ch], y = a.target[3 * pix + ch];
  const float sgn = x > y ? 1.f : (x < y ? -1.f : 0.f);
  const float dmean = f[0] + 2.f * x * f[1] + y * f[2];
  const float sc = lv.scale[w.v];
  a.dL[3 * pix + ch] = sc * ((1.f - a.lambda) * sgn - a.lambda * dmean);
}

// Sum of the tile shares in a fixed order: one block, strided partial sums,
// then a tree over the block.
__global__ __launch_bounds__(256) void loss_finalize(const double* part, int64_t n, float* loss) {
  __shared__ double s_red[4];
  double s = 0.0;
  // unrolled so that a thread's loads are in flight together (same order of additions)
#pragma unroll 8
  for (int64_t k = threadIdx.x; k < n; k += 256) s += part[k];
  s = block_sum_256(s, s_red);
  if (threadIdx.x == 0) *loss = static_cast<float>(s);
}

// Adam with bias correction; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ __launch_bounds__(256) void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n,
                                                   float lr, AdamStep as) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < n; k += stride) {
    float mk = m[k], vk = v[k];
    p[k] = adam_update(p[k], g[k], mk, vk, lr, as);
    m[k] = mk;
    v[k] = vk;
  }
}

// Taps of the normalised 11-tap Gaussian window (sigma 1.5), in double then
// rounded once.
void gauss_taps(float* g) {
  double sum = 0.0, gd[11];
  for (int k = 0; k < 11; ++k) {
    const double d = k - 5;
    gd[k] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
    sum += gd[k];
  }
  for (int k = 0; k < 11; ++k) g[k] = static_cast<float>(gd[k] / sum);
}

}  // namespace

int64_t loss_tiles(const wsr_camera* cams, int32_t nv) {
  int64_t t = 0;
  for (int v = 0; v < nv; ++v)
    t += static_cast<int64_t>((cams[v].width + kLT - 1) / kLT) * ((cams[v].height + kLT - 1) / kLT);
  return t;
}

int64_t loss_workspace_bytes(const wsr_camera* cams, int32_t nv) {
  int64_t pixels = 0;
  for (int v = 0; v < nv; ++v) pixels += static_cast<int64_t>(cams[v].width) * cams[v].height;
  const int64_t maps = (sizeof(float) * 9 * pixels + 255) / 256 * 256;
  return maps + static_cast<int64_t>(sizeof(double)) * 3 * loss_tiles(cams, nv);
}

hipError_t launch_loss(const wsr_camera* cams, int32_t nv, const float* img, const float* target, float lambda,
                       void* ws, float* loss, float* dL, hipStream_t st) {
  hipError_t e = hipSuccess;
  int64_t pixels = 0;
  for (int v = 0; v < nv; ++v) pixels += static_cast<int64_t>(cams[v].width) * cams[v].height;
  LossArgs a;
  a.img = img;
  a.target = target;
  a.dmaps = static_cast<float*>(ws);
  a.part = reinterpret_cast<double*>(static_cast<char*>(ws) + (sizeof(float) * 9 * pixels + 255) / 256 * 256);
  a.dL = dL;
  a.total_pixels = pixels;
  a.lambda = lambda;
  int64_t pix_base = 0;
  int32_t tile0 = 0;
  for (int v0 = 0; v0 < nv; v0 += kLossViewsPerLaunch) {
    LossViews lv = {};
    gauss_taps(lv.gauss);
    lv.nv = nv - v0 < kLossViewsPerLaunch ? nv - v0 : kLossViewsPerLaunch;
    lv.tile0 = tile0;
    int32_t tiles = 0;
    for (int k = 0; k < lv.nv; ++k) {
      const wsr_camera& c = cams[v0 + k];
      lv.width[k] = c.width;
      lv.height[k] = c.height;
      lv.tiles_x[k] = (c.width + kLT - 1) / kLT;
      lv.tile_base[k] = tiles;
      lv.pix_base[k] = pix_base;
      lv.scale[k] = static_cast<float>(1.0 / (3.0 * c.width * c.height * nv));
      tiles += lv.tiles_x[k] * ((c.height + kLT - 1) / kLT);
      pix_base += static_cast<int64_t>(c.width) * c.height;
    }
    lv.tile_base[lv.nv] = tiles;
    if (tiles > 0) {
      loss_pass1<<<dim3(static_cast<unsigned>(tiles), 3), 256, 0, st>>>(a, lv);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    tile0 += tiles;
  }
  pix_base = 0;
  tile0 = 0;
  for (int v0 = 0; v0 < nv; v0 += kLossViewsPerLaunch) {
    LossViews lv = {};
    gauss_taps(lv.gauss);
    lv.nv = nv - v0 < kLossViewsPerLaunch ? nv - v0 : kLossViewsPerLaunch;
    lv.tile0 = tile0;
    int32_t tiles = 0;
    for (int k = 0; k < lv.nv; ++k) {
      const wsr_camera& c = cams[v0 + k];
      lv.width[k] = c.width;
      lv.height[k] = c.height;
      lv.tiles_x[k] = (c.width + kLT - 1) / kLT;
      lv.tile_base[k] = tiles;
      lv.pix_base[k] = pix_base;
      lv.scale[k] = static_cast<float>(1.0 / (3.0 * c.width * c.height * nv));
      tiles += lv.tiles_x[k] * ((c.height + kLT - 1) / kLT);
      pix_base += static_cast<int64_t>(c.width) * c.height;
    }
    lv.tile_base[lv.nv] = tiles;
    if (tiles > 0) {
      loss_pass2<<<dim3(static_cast<unsigned>(tiles), 3), 256, 0, st>>>(a, lv);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    tile0 += tiles;
  }
  loss_finalize<<<1, 256, 0, st>>>(a.part, static_cast<int64_t>(tile0) * 3, loss);
  return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t loss_static_workspace(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidValue;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int32_t step, float lr, float b1,
                       float b2, float eps, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  adam_kernel<<<static_cast<unsigned>(blocks), 256, 0, st>>>(p, g, m, v, n, lr, make_adam_step(step, b1, b2, eps));
  return hipGetLastError();
}

}  // namespace wsr
