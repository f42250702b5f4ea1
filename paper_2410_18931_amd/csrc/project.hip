// Steps a1-a5 of the WSR path: per (view, Gaussian) projection (Sec. 3,
// Eqs. 3-5), SH colour (Eq. 4), maximum opacity (logit, or the unclamped SH
// opacity of Sec. 4.3, Eq. 11), depth weight (Sec. 4.2, Eqs. 8-10) and the
// tile rectangle covered by the support ellipse q <= tau.
//
// One thread per Gaussian, looping over the views, so each Gaussian's
// attributes are read from HBM once per launch with coalesced planar loads.
// The geometry (view transform, Jacobian, Sigma2D, its inverse and the
// projected centre) is evaluated in double precision: at 1080p the centre
// lands up to ~1000 px from the principal point and a float32 evaluation
// moves it by ~1e-4 px, which alone exceeds the image tolerance for the
// smallest splats.  MI355X runs FP64 vector code at half the FP32 packed
// rate, and this kernel is bound by HBM reads, so the cost is hidden.
#include "geom.h"
#include "sh_basis.h"
#include "wsr_internal.h"

namespace wsr {
namespace {

struct ProjArgs {
  const void* means;
  const void* log_scales;
  const void* quats;
  const void* sh;
  const float* logit;
  const float* lc_v;
  const float* globals;
  const DevCamera* cams;
  DevSplat* rec;
  uint2* rect;
  float* out_proj;
  int64_t n;
  int32_t nv;
  int32_t opa_mode;
  int32_t weight_kind;
  int32_t tile;
  float tau, dilation, near_z, opacity_offset, alpha_cut;
  int32_t oit;
};

// float -> fp16 bits, rounded towards +inf (the support extents must never
// shrink); values beyond the fp16 range become +inf.
__device__ inline uint32_t half_bits_up(float x) {
  _Float16 h = static_cast<_Float16>(x);
  uint16_t b = __builtin_bit_cast(uint16_t, h);
  if (static_cast<float>(h) < x) b = static_cast<uint16_t>(b + 1);
  return b;
}

// ONE: a single view.  The colour and opacity are evaluated first, from the
// direction to the camera centre, so the SH coefficients are dead before the
// FP64 geometry needs its registers (one view needs them only once); with
// several views the coefficients stay live across the view loop.
template <int S, int DEG, bool ONE>
__global__ __launch_bounds__(kProjBlock) void project_kernel(ProjArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kProjBlock + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  constexpr int K = (DEG + 1) * (DEG + 1);

  // ---- a1: load and activate attributes (planar SoA, coalesced) ----
  const double p0 = load_attr<S>(a.means, i);
  const double p1 = load_attr<S>(a.means, n + i);
  const double p2 = load_attr<S>(a.means, 2 * n + i);
  QuatScale qs;
  const Sigma3 S3 = make_sigma3(load_attr<S>(a.quats, i), load_attr<S>(a.quats, n + i),
                                load_attr<S>(a.quats, 2 * n + i), load_attr<S>(a.quats, 3 * n + i),
                                load_attr<S>(a.log_scales, i), load_attr<S>(a.log_scales, n + i),
                                load_attr<S>(a.log_scales, 2 * n + i), &qs);
  float4 coef[K];
#pragma unroll
  for (int k = 0; k < K; ++k) coef[k] = load_attr4<S>(a.sh, k * n + i);
  const float logit = a.opa_mode == WSR_OPACITY_LOGIT ? a.logit[i] : 0.f;
  const float lcv = a.weight_kind == WSR_WEIGHT_LC ? a.lc_v[i] : 0.f;
  const float sigma = a.globals[0], beta = a.globals[1];

  const int nv = ONE ? 1 : a.nv;
  for (int v = 0; v < nv; ++v) {
    const DevCamera& cam = a.cams[v];
    const int64_t slot = static_cast<int64_t>(v) * n + i;
    // ---- a4: SH colour and opacity at the view direction ----
    double dir[3], len;
    view_dir_cam(cam, p0, p1, p2, dir, &len);
    float rgb[3], u;
    {
      float Y[K];
      sh_eval<DEG>(static_cast<float>(dir[0]), static_cast<float>(dir[1]), static_cast<float>(dir[2]), Y);
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        acc.x = fmaf(coef[k].x, Y[k], acc.x);
        acc.y = fmaf(coef[k].y, Y[k], acc.y);
        acc.z = fmaf(coef[k].z, Y[k], acc.z);
        acc.w = fmaf(coef[k].w, Y[k], acc.w);
      }
      rgb[0] = fmaxf(acc.x + 0.5f, 0.f);
      rgb[1] = fmaxf(acc.y + 0.5f, 0.f);
      rgb[2] = fmaxf(acc.z + 0.5f, 0.f);
      u = a.opa_mode == WSR_OPACITY_SH ? acc.w + a.opacity_offset : 1.f / (1.f + expf(-logit));
    }
    // ---- opacity early-out (App. D; off with alpha_cut = 0): a pair
    // contributes only while u exp(-q/2) >= alpha_cut, i.e. while
    // q <= 2 ln(u / alpha_cut); a Gaussian with u <= alpha_cut never does.
    // The cutoff is a support decision, so u is evaluated again in double
    // precision for it (the float32 u above carries the SH sum's rounding,
    // which would move the cutoff by far more than the float rounding of
    // q); the only float32 step left is the rounding of the cutoff itself.
    double u64 = 0.0;
    if (a.alpha_cut > 0.f) {
      if (a.opa_mode == WSR_OPACITY_SH) {
        double Y64[K];
        sh_eval_f64<DEG>(dir[0], dir[1], dir[2], Y64);
        u64 = a.opacity_offset;
#pragma unroll
        for (int k = 0; k < K; ++k) u64 = fma(static_cast<double>(coef[k].w), Y64[k], u64);
      } else {
        u64 = 1.0 / (1.0 + exp(-static_cast<double>(logit)));
      }
    }
    // ---- a2, a3: view transform, cull, EWA ----
    ViewGeom g;
    const bool vis = view_geom(cam, p0, p1, p2, S3, qs.ok, a.near_z, a.dilation, &g);
    float w = 0.f;
    uint2 rect = make_uint2(0u, 0u);
    bool alive = vis;
    if (!vis) {
      rgb[0] = rgb[1] = rgb[2] = 0.f;
      u = 0.f;
    }
    if (vis) {
      // ---- a5: depth weight ----
      const float d = static_cast<float>(g.tz);
      if (a.weight_kind == WSR_WEIGHT_DIR) {
        w = 1.f;
      } else if (a.weight_kind == WSR_WEIGHT_EXP) {
        w = expf(-sigma * powf(d, beta));
      } else {
        w = fmaxf(1.f - d / sigma, 0.f) * lcv;
      }
      double cut = a.tau;
      if (a.alpha_cut > 0.f) {
        alive = u64 > a.alpha_cut;
        if (alive) cut = fmin(cut, 2.0 * log(u64 / static_cast<double>(a.alpha_cut)));
      }
    // ---- support box of q <= cut, widened so float rounding of q never
      // reaches a pixel outside it ----
      const double ex = sqrt(cut * g.c00) * (1.0 + 1e-4) + 1e-3;
      const double ey = sqrt(cut * g.c11) * (1.0 + 1e-4) + 1e-3;
      const double plo_x = ceil(g.mux - ex - 0.5), phi_x = floor(g.mux + ex - 0.5);
      const double plo_y = ceil(g.muy - ey - 0.5), phi_y = floor(g.muy + ey - 0.5);
      if (alive && phi_x >= 0.0 && plo_x <= cam.width - 1.0 && phi_y >= 0.0 && plo_y <= cam.height - 1.0) {
        const int T = a.tile;
        const int x0 = static_cast<int>(fmax(plo_x, 0.0)) / T;
        const int x1 = static_cast<int>(fmin(phi_x, cam.width - 1.0)) / T + 1;
        const int y0 = static_cast<int>(fmax(plo_y, 0.0)) / T;
        const int y1 = static_cast<int>(fmin(phi_y, cam.height - 1.0)) / T + 1;
        rect = make_uint2(static_cast<uint32_t>(x0) | (static_cast<uint32_t>(x1) << 16),
                          static_cast<uint32_t>(y0) | (static_cast<uint32_t>(y1) << 16));
      }
      const double ox = floor(g.mux), oy = floor(g.muy);
      SplatRec r;
      r.r0 = make_float4(static_cast<float>(g.mux - ox), static_cast<float>(g.muy - oy),
                         static_cast<float>(g.A), static_cast<float>(2.0 * g.B));
      r.r1 = make_float4(static_cast<float>(g.C), static_cast<float>(ox), static_cast<float>(oy), u * w);
      // the fourth word: the support half-extents for culling, or with the
      // early-out the splat's own cutoff (the raster then derives the
      // extents from the conic)
      const uint32_t ext = half_bits_up(static_cast<float>(ex)) | (half_bits_up(static_cast<float>(ey)) << 16);
      r.r2 = make_float4(rgb[0], rgb[1], rgb[2], a.alpha_cut > 0.f ? static_cast<float>(cut) : __uint_as_float(ext));
      DevSplat ds;
      ds.s = r;
      // the tile rectangle locates a pair's Gaussian-major slot; the camera
      // depth orders the splats for the sorted-blending baseline, the
      // opacity enters Eq. 2's coverage term in OIT mode (the first word is
      // unused)
      ds.slot = make_uint4(0u, rect.x, rect.y, __float_as_uint(a.oit ? u : static_cast<float>(g.tz)));
      a.rec[slot] = ds;
    }
    a.rect[slot] = rect;
    if (a.out_proj) {
      float4* o = reinterpret_cast<float4*>(a.out_proj + slot * 16);
      o[0] = make_float4(alive ? 1.f : 0.f, vis ? static_cast<float>(g.mux) : 0.f,
                         vis ? static_cast<float>(g.muy) : 0.f, vis ? static_cast<float>(g.A) : 0.f);
      o[1] = make_float4(vis ? static_cast<float>(g.B) : 0.f, vis ? static_cast<float>(g.C) : 0.f, rgb[0], rgb[1]);
      o[2] = make_float4(rgb[2], u, w, static_cast<float>(g.tz));
      o[3] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

template <int S, bool ONE>
void launch_sd(const ProjArgs& a, int deg, dim3 grid, hipStream_t st) {
  switch (deg) {
    case 0: project_kernel<S, 0, ONE><<<grid, kProjBlock, 0, st>>>(a); break;
    case 1: project_kernel<S, 1, ONE><<<grid, kProjBlock, 0, st>>>(a); break;
    case 2: project_kernel<S, 2, ONE><<<grid, kProjBlock, 0, st>>>(a); break;
    default: project_kernel<S, 3, ONE><<<grid, kProjBlock, 0, st>>>(a); break;
  }
}

template <int S>
hipError_t launch_s(const ProjArgs& a, int deg, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((a.n + kProjBlock - 1) / kProjBlock));
  if (a.nv == 1)
    launch_sd<S, true>(a, deg, grid, st);
  else
    launch_sd<S, false>(a, deg, grid, st);
  return hipGetLastError();
}

// Cameras reach the device as a kernel argument (no host-memory copy, so the
// upload is capturable in a graph); 16 per launch keeps the argument < 4 KB.
constexpr int kCamsPerUpload = 16;
struct CamBatch {
  DevCamera c[kCamsPerUpload];
  int32_t count;
  int32_t first;
};
__global__ void upload_cameras_kernel(CamBatch b, DevCamera* dst) {
  const int k = threadIdx.x;
  if (k < b.count) dst[b.first + k] = b.c[k];
}

}  // namespace

hipError_t launch_upload_cameras(const DevCamera* dc, int32_t nv, void* ws, const Layout& L,
                                 hipStream_t st) {
  DevCamera* dst = at<DevCamera>(ws, L.off_cams);
  for (int first = 0; first < nv; first += kCamsPerUpload) {
    CamBatch b;
    b.count = nv - first < kCamsPerUpload ? nv - first : kCamsPerUpload;
    b.first = first;
    for (int k = 0; k < b.count; ++k) b.c[k] = dc[first + k];
    upload_cameras_kernel<<<1, kCamsPerUpload, 0, st>>>(b, dst);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_project(const wsr_scene* sc, const wsr_params* P, const float* globals,
                          const Layout& L, void* ws, float* out_proj, hipStream_t st) {
  if (L.n == 0) return hipSuccess;
  ProjArgs a;
  a.means = sc->means;
  a.log_scales = sc->log_scales;
  a.quats = sc->quats;
  a.sh = sc->sh;
  a.logit = sc->opacity_logit;
  a.lc_v = sc->lc_v;
  a.globals = globals;
  a.cams = at<DevCamera>(ws, L.off_cams);
  a.rec = at<DevSplat>(ws, L.off_rec);
  a.rect = at<uint2>(ws, L.off_rect);
  a.out_proj = out_proj;
  a.n = L.n;
  a.nv = L.nv;
  a.opa_mode = sc->opacity_mode;
  a.weight_kind = P->weight_kind;
  a.tile = P->tile;
  a.tau = P->tau;
  a.alpha_cut = P->alpha_cut;
  a.oit = (P->flags & WSR_FLAG_OIT) ? 1 : 0;
  a.dilation = P->dilation;
  a.near_z = P->near_z;
  a.opacity_offset = P->opacity_offset;
  switch (sc->storage) {
    case WSR_STORE_F16: return launch_s<WSR_STORE_F16>(a, sc->sh_degree, st);
    case WSR_STORE_BF16: return launch_s<WSR_STORE_BF16>(a, sc->sh_degree, st);
    default: return launch_s<WSR_STORE_F32>(a, sc->sh_degree, st);
  }
}

}  // namespace wsr
