// Step a9 of the WSR path: chain the per-(view, Gaussian) 2D gradients
// (dL/d mu, conic, colour, amplitude) back to the scene parameters of Sec. 3
// (centre, log-scale, quaternion, SH), the opacity (logit, or the SH opacity
// of Sec. 4.3, Eq. 11), the depth-weight parameters (Eqs. 9, 10) and the
// background weight and colour of Eq. 7.
//
// One thread per Gaussian, looping over the views, so no atomics are needed
// and every gradient is written once with coalesced planar stores.  The
// gradient of Sigma3D is summed over views first and chained to (q, s) once.
// The global parameters are reduced in double precision from per-block
// partials (deterministic, no float atomics).
#include "adam.h"
#include "geom.h"
#include "sh_basis.h"
#include "wsr_internal.h"

namespace wsr {
namespace {

constexpr int kBwdBlock = 128;

struct BwdArgs {
  const void* means;
  const void* log_scales;
  const void* quats;
  const void* sh;
  const float* logit;
  const float* lc_v;
  const float* globals;
  const DevCamera* cams;
  const float* grad2d;       // per-(view, Gaussian) 2D gradients [nv][n][9]
  const float* du2d;         // OIT: per-(view, Gaussian) dL/du of Eq. 2's coverage term, else null
  wsr_grads g;
  double* gpart;      // [blocks][2] = sigma, beta
  int64_t n;
  int32_t nv;
  int32_t opa_mode;
  int32_t weight_kind;
  float near_z, dilation, opacity_offset;
  // ADAM instances: the FP32 parameters (updated in place), the moments in
  // the gradients' layout and one learning rate per group (means,
  // log-scales, quaternions, SH degree 0, higher SH degrees, logit, v_i)
  float* p_means;
  float* p_log_scales;
  float* p_quats;
  float* p_sh;
  float* p_logit;
  float* p_lc_v;
  wsr_grads m, v;
  float lr[7];
  AdamStep as;
};

// The parameter's new value, its moments updated in place (see adam.h).
__device__ __forceinline__ void adam_store(float* p, float* m, float* v, int64_t o, float pv, float g, float mk,
                                           float vk, float lr, const AdamStep& s) {
  p[o] = adam_update(pv, g, mk, vk, lr, s);
  m[o] = mk;
  v[o] = vk;
}

// ADAM: instead of writing the per-Gaussian gradients, apply one Adam step to
// the parameters with them (the values the plain instance writes, so both
// paths give the same bits); the moments are read up front, before any
// store, so that their loads are in flight together.
template <int S, int DEG, bool ADAM>
__global__ __launch_bounds__(kBwdBlock) void project_bwd_kernel(BwdArgs a) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ double s_red[kBwdBlock / kWave][2];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBwdBlock + threadIdx.x;
  const int64_t n = a.n;
  double gsig = 0.0, gbeta = 0.0;
  if (i < n) {
    // Every load of the attributes and of the first view's 2D gradient is
    // issued before any arithmetic (the scheduling barrier keeps them
    // together), so each thread pays one memory round trip up front.
    const float m0 = load_attr<S>(a.means, i), m1 = load_attr<S>(a.means, n + i),
                m2 = load_attr<S>(a.means, 2 * n + i);
    const float rq[4] = {load_attr<S>(a.quats, i), load_attr<S>(a.quats, n + i),
                         load_attr<S>(a.quats, 2 * n + i), load_attr<S>(a.quats, 3 * n + i)};
    const float l0 = load_attr<S>(a.log_scales, i), l1 = load_attr<S>(a.log_scales, n + i),
                l2 = load_attr<S>(a.log_scales, 2 * n + i);
    float4 coef[K];
#pragma unroll
    for (int k = 0; k < K; ++k) coef[k] = load_attr4<S>(a.sh, k * n + i);
    const float logit = a.opa_mode == WSR_OPACITY_LOGIT ? a.logit[i] : 0.f;
    const float lcv = a.weight_kind == WSR_WEIGHT_LC ? a.lc_v[i] : 0.f;
    float gv0[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) gv0[j] = a.grad2d[i * 9 + j];
    __builtin_amdgcn_sched_barrier(0);
    const double p0 = m0, p1 = m1, p2 = m2;
    QuatScale qs;
    const Sigma3 S3 = make_sigma3(rq[0], rq[1], rq[2], rq[3], l0, l1, l2, &qs);
    const double sigma = a.globals[0], beta = a.globals[1];

    double dp[3] = {0.0, 0.0, 0.0};
    double dS[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // symmetric dL/dSigma3D (xx, xy, xz, yy, yz, zz)
    float4 dsh[K];
#pragma unroll
    for (int k = 0; k < K; ++k) dsh[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    float dlogit = 0.f, dv = 0.f;

    // View v's 2D gradient (and OIT dL/du) comes from gn, which the previous
    // iteration requested: with one wave per SIMD, loading it at the top of
    // its own iteration would expose a memory round trip per view.
    float gn[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) gn[j] = gv0[j];
    float dn = a.du2d ? a.du2d[i] : 0.f;
    for (int v = 0; v < a.nv; ++v) {
      float gv[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) gv[j] = gn[j];
      const float du_cov = dn;
      if (v + 1 < a.nv) {
        const float* g2 = a.grad2d + (static_cast<int64_t>(v + 1) * n + i) * 9;
#pragma unroll
        for (int j = 0; j < 9; ++j) gn[j] = g2[j];
        if (a.du2d) dn = a.du2d[static_cast<int64_t>(v + 1) * n + i];
      }
      bool nz = du_cov != 0.f;
#pragma unroll
      for (int j = 0; j < 9; ++j) nz |= gv[j] != 0.f;
      if (!nz) continue;
      const DevCamera& cam = a.cams[v];
      ViewGeom g;
      if (!view_geom(cam, p0, p1, p2, S3, qs.ok, a.near_z, a.dilation, &g)) continue;
      double dt[3] = {0.0, 0.0, 0.0};

      // --- colour, opacity and weight (a4, a5) ---
      double dir[3], len;
      view_dir(g, cam, p0, p1, p2, dir, &len);
      const float fx3 = static_cast<float>(dir[0]), fy3 = static_cast<float>(dir[1]), fz3 = static_cast<float>(dir[2]);
      float Y[K];
      sh_eval<DEG>(fx3, fy3, fz3, Y);
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        acc.x = fmaf(coef[k].x, Y[k], acc.x);
        acc.y = fmaf(coef[k].y, Y[k], acc.y);
        acc.z = fmaf(coef[k].z, Y[k], acc.z);
        acc.w = fmaf(coef[k].w, Y[k], acc.w);
      }
      const float u = a.opa_mode == WSR_OPACITY_SH ? acc.w + a.opacity_offset : 1.f / (1.f + expf(-logit));
      const double d = g.tz;
      double w = 1.0, dw_dd = 0.0;
      if (a.weight_kind == WSR_WEIGHT_EXP) {
        const double db = pow(d, beta);
        w = exp(-sigma * db);
        dw_dd = -sigma * beta * db / d * w;
      } else if (a.weight_kind == WSR_WEIGHT_LC) {
        const double lin = 1.0 - d / sigma;
        w = lin > 0.0 ? lin * lcv : 0.0;
        dw_dd = lin > 0.0 ? -lcv / sigma : 0.0;
      }
      const double gamp = gv[8];
      // u enters the amplitude u w and, in OIT mode, the coverage term
      const double du = gamp * w + du_cov, dw = gamp * u;
      if (a.weight_kind == WSR_WEIGHT_EXP) {
        const double db = pow(d, beta);
        gsig += dw * (-db * w);
        gbeta += dw * (-sigma * db * log(d) * w);
      } else if (a.weight_kind == WSR_WEIGHT_LC) {
        const double lin = 1.0 - d / sigma;
        if (lin > 0.0) {
          dv += static_cast<float>(dw * lin);
          gsig += dw * lcv * d / (sigma * sigma);
        }
      }
      dt[2] += dw * dw_dd;
      // gradient at the raw (pre-activation) SH sums, RGBA
      float4 graw;
      graw.x = acc.x + 0.5f > 0.f ? gv[5] : 0.f;
      graw.y = acc.y + 0.5f > 0.f ? gv[6] : 0.f;
      graw.z = acc.z + 0.5f > 0.f ? gv[7] : 0.f;
      graw.w = 0.f;
      if (a.opa_mode == WSR_OPACITY_SH) graw.w = static_cast<float>(du);
      else dlogit += static_cast<float>(du) * u * (1.f - u);
      float3 gY[K];
      sh_eval_grad<DEG>(fx3, fy3, fz3, gY);
      float3 ddir = make_float3(0.f, 0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        dsh[k].x = fmaf(graw.x, Y[k], dsh[k].x);
        dsh[k].y = fmaf(graw.y, Y[k], dsh[k].y);
        dsh[k].z = fmaf(graw.z, Y[k], dsh[k].z);
        dsh[k].w = fmaf(graw.w, Y[k], dsh[k].w);
        const float c = coef[k].x * graw.x + coef[k].y * graw.y + coef[k].z * graw.z + coef[k].w * graw.w;
        ddir.x = fmaf(c, gY[k].x, ddir.x);
        ddir.y = fmaf(c, gY[k].y, ddir.y);
        ddir.z = fmaf(c, gY[k].z, ddir.z);
      }
      {
        const double dd3[3] = {ddir.x, ddir.y, ddir.z};
        const double radial = dd3[0] * dir[0] + dd3[1] * dir[1] + dd3[2] * dir[2];
        for (int c = 0; c < 3; ++c) dp[c] += (dd3[c] - radial * dir[c]) / len;
      }

      // --- projected centre ---
      const double gmx = gv[0], gmy = gv[1];
      const double fx = cam.fx, fy = cam.fy, iz = g.izt;
      dt[0] += gmx * fx * iz;
      dt[1] += gmy * fy * iz;
      dt[2] -= (gmx * fx * g.tx + gmy * fy * g.ty) * iz * iz;

      // --- conic -> Sigma2D: dL/dSigma = -Q G Q with G the symmetric
      // gradient of the conic matrix Q = [[A, B], [B, C]] ---
      const double gA = gv[2], gBh = 0.5 * gv[3], gC = gv[4];
      const double P00 = gA * g.A + gBh * g.B, P01 = gA * g.B + gBh * g.C;
      const double P10 = gBh * g.A + gC * g.B, P11 = gBh * g.B + gC * g.C;
      const double GS00 = -(g.A * P00 + g.B * P10);
      const double GS11 = -(g.B * P01 + g.C * P11);
      const double GS01 = -0.5 * ((g.A * P01 + g.B * P11) + (g.B * P00 + g.C * P10));

      // --- Sigma2D = Tm S Tm^T + dilation, Tm rows a, b ---
      double Sa[3], Sb[3];
      sym_mul(S3, g.a, Sa);
      sym_mul(S3, g.b, Sb);
      // dL/dS += Tm^T G Tm
      const double* A3 = g.a;
      const double* B3 = g.b;
      dS[0] += GS00 * A3[0] * A3[0] + 2.0 * GS01 * A3[0] * B3[0] + GS11 * B3[0] * B3[0];
      dS[1] += GS00 * A3[0] * A3[1] + GS01 * (A3[0] * B3[1] + B3[0] * A3[1]) + GS11 * B3[0] * B3[1];
      dS[2] += GS00 * A3[0] * A3[2] + GS01 * (A3[0] * B3[2] + B3[0] * A3[2]) + GS11 * B3[0] * B3[2];
      dS[3] += GS00 * A3[1] * A3[1] + 2.0 * GS01 * A3[1] * B3[1] + GS11 * B3[1] * B3[1];
      dS[4] += GS00 * A3[1] * A3[2] + GS01 * (A3[1] * B3[2] + B3[1] * A3[2]) + GS11 * B3[1] * B3[2];
      dS[5] += GS00 * A3[2] * A3[2] + 2.0 * GS01 * A3[2] * B3[2] + GS11 * B3[2] * B3[2];
      // dL/dTm = 2 G Tm S
      double ga[3], gb[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        ga[j] = 2.0 * (GS00 * Sa[j] + GS01 * Sb[j]);
        gb[j] = 2.0 * (GS01 * Sa[j] + GS11 * Sb[j]);
      }
      // a_j = fx/tz (W0j - rx W2j), b_j = fy/tz (W1j - ry W2j), rx = tx/tz unless clamped
      const double* W = g.W;
      const double ex = g.unclamped_x ? 1.0 : 0.0, ey = g.unclamped_y ? 1.0 : 0.0;
      const double kx = fx * iz * iz, ky = fy * iz * iz;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        dt[2] -= ga[j] * kx * (W[j] - (1.0 + ex) * g.rx * W[6 + j]);
        dt[2] -= gb[j] * ky * (W[3 + j] - (1.0 + ey) * g.ry * W[6 + j]);
        dt[0] -= ex * ga[j] * kx * W[6 + j];
        dt[1] -= ey * gb[j] * ky * W[6 + j];
      }
      // t = W p + T
#pragma unroll
      for (int c = 0; c < 3; ++c) dp[c] += W[c] * dt[0] + W[3 + c] * dt[1] + W[6 + c] * dt[2];
    }

    // --- Sigma3D = M M^T, M = R diag(s): dL/dM = 2 G M ---
    const double* R = qs.R;
    const double s[3] = {qs.s0, qs.s1, qs.s2};
    const double G[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
    double gR[9], gs[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double gM = 2.0 * (G[3 * r] * R[j] * s[j] + G[3 * r + 1] * R[3 + j] * s[j] + G[3 * r + 2] * R[6 + j] * s[j]);
        gR[3 * r + j] = gM * s[j];
        gs[j] += gM * R[3 * r + j];
      }
    // R = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]x for the unit quaternion (w, v)
    const double w = qs.w, x = qs.x, y = qs.y, z = qs.z;
    const double tr = gR[0] + gR[4] + gR[8];
    const double kxs = gR[7] - gR[5], kys = gR[2] - gR[6], kzs = gR[3] - gR[1];
    double gq[4];
    gq[0] = 2.0 * w * tr + 2.0 * (x * kxs + y * kys + z * kzs);
    const double vv[3] = {x, y, z};
    const double ks[3] = {kxs, kys, kzs};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double Gv = gR[3 * c] * x + gR[3 * c + 1] * y + gR[3 * c + 2] * z;   // (G v)_c
      const double GTv = gR[c] * x + gR[3 + c] * y + gR[6 + c] * z;              // (G^T v)_c
      gq[1 + c] = -2.0 * vv[c] * tr + 2.0 * (Gv + GTv) + 2.0 * w * ks[c];
    }
    // through q / |q|
    const double qn = sqrt(static_cast<double>(rq[0]) * rq[0] + static_cast<double>(rq[1]) * rq[1] +
                           static_cast<double>(rq[2]) * rq[2] + static_cast<double>(rq[3]) * rq[3]);
    const double qh[4] = {w, x, y, z};
    const double proj = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;

    const bool ok = qs.ok;
    float gm[3], gl[3], gqt[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) gm[c] = static_cast<float>(dp[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) gl[c] = ok ? static_cast<float>(gs[c] * s[c]) : 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) gqt[c] = ok ? static_cast<float>((gq[c] - qh[c] * proj) / qn) : 0.f;
    if (ADAM) {
      const bool upd_logit = a.p_logit && a.m.opacity_logit && a.v.opacity_logit;
      const bool upd_lcv = a.p_lc_v && a.m.lc_v && a.v.lc_v;
      float mm[10], vm[10];
      float4 msh[K], vsh[K];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mm[c] = a.m.means[c * n + i];
        vm[c] = a.v.means[c * n + i];
        mm[3 + c] = a.m.log_scales[c * n + i];
        vm[3 + c] = a.v.log_scales[c * n + i];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        mm[6 + c] = a.m.quats[c * n + i];
        vm[6 + c] = a.v.quats[c * n + i];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        msh[k] = reinterpret_cast<const float4*>(a.m.sh)[k * n + i];
        vsh[k] = reinterpret_cast<const float4*>(a.v.sh)[k * n + i];
      }
      // the logit and v_i values were read above only where the modes use them
      const float pl = upd_logit ? (a.opa_mode == WSR_OPACITY_LOGIT ? logit : a.p_logit[i]) : 0.f;
      const float ml = upd_logit ? a.m.opacity_logit[i] : 0.f, vl = upd_logit ? a.v.opacity_logit[i] : 0.f;
      const float pv = upd_lcv ? (a.weight_kind == WSR_WEIGHT_LC ? lcv : a.p_lc_v[i]) : 0.f;
      const float mv = upd_lcv ? a.m.lc_v[i] : 0.f, vv = upd_lcv ? a.v.lc_v[i] : 0.f;
      const float pmean[3] = {m0, m1, m2}, plog[3] = {l0, l1, l2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        adam_store(a.p_means, a.m.means, a.v.means, c * n + i, pmean[c], gm[c], mm[c], vm[c], a.lr[0], a.as);
        adam_store(a.p_log_scales, a.m.log_scales, a.v.log_scales, c * n + i, plog[c], gl[c], mm[3 + c],
                   vm[3 + c], a.lr[1], a.as);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
        adam_store(a.p_quats, a.m.quats, a.v.quats, c * n + i, rq[c], gqt[c], mm[6 + c], vm[6 + c], a.lr[2], a.as);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float lr = k == 0 ? a.lr[3] : a.lr[4];
        float4 p4 = coef[k], m4 = msh[k], v4 = vsh[k];
        p4.x = adam_update(p4.x, dsh[k].x, m4.x, v4.x, lr, a.as);
        p4.y = adam_update(p4.y, dsh[k].y, m4.y, v4.y, lr, a.as);
        p4.z = adam_update(p4.z, dsh[k].z, m4.z, v4.z, lr, a.as);
        p4.w = adam_update(p4.w, dsh[k].w, m4.w, v4.w, lr, a.as);
        reinterpret_cast<float4*>(a.p_sh)[k * n + i] = p4;
        reinterpret_cast<float4*>(a.m.sh)[k * n + i] = m4;
        reinterpret_cast<float4*>(a.v.sh)[k * n + i] = v4;
      }
      if (upd_logit) adam_store(a.p_logit, a.m.opacity_logit, a.v.opacity_logit, i, pl, dlogit, ml, vl, a.lr[5], a.as);
      if (upd_lcv) adam_store(a.p_lc_v, a.m.lc_v, a.v.lc_v, i, pv, dv, mv, vv, a.lr[6], a.as);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.g.means[c * n + i] = gm[c];
#pragma unroll
      for (int c = 0; c < 3; ++c) a.g.log_scales[c * n + i] = gl[c];
#pragma unroll
      for (int c = 0; c < 4; ++c) a.g.quats[c * n + i] = gqt[c];
      float4* gsh = reinterpret_cast<float4*>(a.g.sh);
#pragma unroll
      for (int k = 0; k < K; ++k) gsh[k * n + i] = dsh[k];
      if (a.g.opacity_logit) a.g.opacity_logit[i] = dlogit;
      if (a.g.lc_v) a.g.lc_v[i] = dv;
    }
  }
  // block partials of dL/dsigma, dL/dbeta
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    gsig += __shfl_xor(gsig, d, kWave);
    gbeta += __shfl_xor(gbeta, d, kWave);
  }
  if (lane == 0) {
    s_red[wv][0] = gsig;
    s_red[wv][1] = gbeta;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kBwdBlock / kWave; ++k) t += s_red[k][threadIdx.x];
    a.gpart[static_cast<int64_t>(blockIdx.x) * 2 + threadIdx.x] = t;
  }
}

// Sum of each (view, Gaussian)'s per-tile partial 2D gradients: its pairs
// occupy a contiguous range of Gaussian-major slots.  A light kernel of its
// own, so the register-heavy chain below reads one 9-float gradient per
// slot.  A lane sums the range of its own Gaussian when it is short; a long
// range (a splat covering many tiles) is summed by the whole wave, lanes
// striding through it, so the largest splats do not form a serial tail.
// With OIT (DU) the same pass also sums each pair's dL/du through the
// coverage term, which the raster stores in an array of its own.
constexpr uint32_t kHeavySlots = 32;

__device__ __forceinline__ void add3(float* g, int o, const float3 v) {
  g[o] += v.x;
  g[o + 1] += v.y;
  g[o + 2] += v.z;
}

template <bool DU>
__global__ __launch_bounds__(256) void sum_pair_partials(const uint32_t* goff, const float3* part, const float* du,
                                                         uint32_t capacity, int64_t slots, float* grad2d,
                                                         float* out_grad2d, float* du2d) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int lane = threadIdx.x % kWave;
  uint32_t s0 = 0, s1 = 0;
  if (k < slots) {
    s0 = goff[k];
    s1 = goff[k + 1];
    s0 = s0 < capacity ? s0 : capacity;
    s1 = s1 < capacity ? s1 : capacity;
    if (s1 < s0) s1 = s0;
  }
  const bool heavy = s1 - s0 > kHeavySlots;
  float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float gu = 0.f;
  if (!heavy) {
    // four slots per step keep twelve loads in flight per lane
    uint32_t j = s0;
    for (; j + 4 <= s1; j += 4) {
      const float3* p = part + 3 * static_cast<int64_t>(j);
      const float3 x0 = p[0], x1 = p[1], x2 = p[2], y0 = p[3], y1 = p[4], y2 = p[5];
      const float3 z0 = p[6], z1 = p[7], z2 = p[8], w0 = p[9], w1 = p[10], w2 = p[11];
      add3(g, 0, x0); add3(g, 3, x1); add3(g, 6, x2);
      add3(g, 0, y0); add3(g, 3, y1); add3(g, 6, y2);
      add3(g, 0, z0); add3(g, 3, z1); add3(g, 6, z2);
      add3(g, 0, w0); add3(g, 3, w1); add3(g, 6, w2);
      if (DU) {
        const float u0 = du[j], u1 = du[j + 1], u2 = du[j + 2], u3 = du[j + 3];
        gu += u0;
        gu += u1;
        gu += u2;
        gu += u3;
      }
    }
    for (; j + 2 <= s1; j += 2) {
      const float3* p = part + 3 * static_cast<int64_t>(j);
      const float3 x0 = p[0], x1 = p[1], x2 = p[2], y0 = p[3], y1 = p[4], y2 = p[5];
      add3(g, 0, x0); add3(g, 3, x1); add3(g, 6, x2);
      add3(g, 0, y0); add3(g, 3, y1); add3(g, 6, y2);
      if (DU) {
        const float u0 = du[j], u1 = du[j + 1];
        gu += u0;
        gu += u1;
      }
    }
    if (j < s1) {
      const float3* p = part + 3 * static_cast<int64_t>(j);
      add3(g, 0, p[0]); add3(g, 3, p[1]); add3(g, 6, p[2]);
      if (DU) gu += du[j];
    }
  }
  // the wave sums its heavy Gaussians one after another
  uint64_t hmask = __ballot(heavy);
  while (hmask) {
    const int src = __ffsll(static_cast<long long>(hmask)) - 1;
    hmask &= hmask - 1;
    const uint32_t h0 = __shfl(s0, src, kWave), h1 = __shfl(s1, src, kWave);
    float w[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (uint32_t j = h0 + lane; j < h1; j += kWave) {
      const float3* p = part + 3 * static_cast<int64_t>(j);
      add3(w, 0, p[0]); add3(w, 3, p[1]); add3(w, 6, p[2]);
      if (DU) w[9] += du[j];
    }
#pragma unroll
    for (int q = 0; q < (DU ? 10 : 9); ++q) {
      float x = w[q];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
      if (lane == src) {
        if (q < 9) g[q] = x;
        else gu = x;
      }
    }
  }
  if (k >= slots) return;
  float* d = grad2d + 9 * k;
#pragma unroll
  for (int q = 0; q < 9; ++q) d[q] = g[q];
  if (out_grad2d) {
#pragma unroll
    for (int q = 0; q < 9; ++q) out_grad2d[9 * k + q] = g[q];
  }
  if (DU) du2d[k] = gu;
}

// Final reduction of the global parameters: dL/dsigma, dL/dbeta from the
// per-block partials, dL/dw_B and dL/dc_B from the per-tile partials.
__global__ __launch_bounds__(1024) void reduce_globals(const double* gpart, int64_t nblocks,
                                                       const float* tilepart, int64_t ntiles, float* out) {
  __shared__ double sh[16][6];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  // unrolled so that a thread's loads are in flight together
#pragma unroll 8
  for (int64_t b = threadIdx.x; b < nblocks; b += 1024) {
    acc[0] += gpart[2 * b];
    acc[1] += gpart[2 * b + 1];
  }
#pragma unroll 8
  for (int64_t t = threadIdx.x; t < ntiles; t += 1024) {
    acc[3] += tilepart[4 * t];
    acc[4] += tilepart[4 * t + 1];
    acc[5] += tilepart[4 * t + 2];
    acc[2] += tilepart[4 * t + 3];
  }
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double x = acc[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    if (lane == 0) sh[wv][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sh[w][threadIdx.x];
    out[threadIdx.x] = static_cast<float>(t);
  }
}

__global__ void fill_zero_kernel(uint32_t* p, int64_t words) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < words; k += stride) p[k] = 0u;
}

template <int S, bool ADAM>
hipError_t bwd_s(const BwdArgs& a, int deg, unsigned blocks, hipStream_t st) {
  switch (deg) {
    case 0: project_bwd_kernel<S, 0, ADAM><<<blocks, kBwdBlock, 0, st>>>(a); break;
    case 1: project_bwd_kernel<S, 1, ADAM><<<blocks, kBwdBlock, 0, st>>>(a); break;
    case 2: project_bwd_kernel<S, 2, ADAM><<<blocks, kBwdBlock, 0, st>>>(a); break;
    default: project_bwd_kernel<S, 3, ADAM><<<blocks, kBwdBlock, 0, st>>>(a); break;
  }
  return hipGetLastError();
}

}  // namespace

int64_t project_bwd_blocks(int64_t n) { return n > 0 ? (n + kBwdBlock - 1) / kBwdBlock : 1; }

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t words = static_cast<int64_t>(bytes / 4);
  if (words == 0) return hipSuccess;
  int64_t blocks = (words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_zero_kernel<<<static_cast<unsigned>(blocks), 256, 0, st>>>(static_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

// The projection backward; with `f` (FP32 storage only) the fused Adam
// instances, which leave the per-Gaussian fields of g unused.
static hipError_t project_bwd_impl(const wsr_scene* sc, const wsr_params* P, const float* globals,
                                   const Layout& L, void* ws, const void* pairs, int64_t capacity,
                                   const wsr_grads* g, const FusedAdam* f, float* out_grad2d, hipStream_t st) {
  double* gpart = at<double>(ws, L.off_gpart);
  const unsigned blocks = static_cast<unsigned>(project_bwd_blocks(L.n));
  hipError_t e = hipSuccess;
  if (L.n > 0) {
    const PairView pv = pair_view(pairs, capacity);
    const int64_t slots = L.n * L.nv;
    const bool oit = (P->flags & WSR_FLAG_OIT) != 0;
    const unsigned sblocks = static_cast<unsigned>((slots + 255) / 256);
    if (oit)
      sum_pair_partials<true><<<sblocks, 256, 0, st>>>(at<uint32_t>(ws, L.off_goff), pv.part, pv.du,
                                                       static_cast<uint32_t>(capacity), slots,
                                                       at<float>(ws, L.off_grad2d), out_grad2d,
                                                       at<float>(ws, L.off_du2d));
    else
      sum_pair_partials<false><<<sblocks, 256, 0, st>>>(at<uint32_t>(ws, L.off_goff), pv.part, nullptr,
                                                        static_cast<uint32_t>(capacity), slots,
                                                        at<float>(ws, L.off_grad2d), out_grad2d, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    BwdArgs a;
    a.means = sc->means;
    a.log_scales = sc->log_scales;
    a.quats = sc->quats;
    a.sh = sc->sh;
    a.logit = sc->opacity_logit;
    a.lc_v = sc->lc_v;
    a.globals = globals;
    a.cams = at<DevCamera>(ws, L.off_cams);
    a.grad2d = at<float>(ws, L.off_grad2d);
    a.du2d = oit ? at<float>(ws, L.off_du2d) : nullptr;
    a.g = *g;
    a.gpart = gpart;
    a.n = L.n;
    a.nv = L.nv;
    a.opa_mode = sc->opacity_mode;
    a.weight_kind = P->weight_kind;
    a.near_z = P->near_z;
    a.dilation = P->dilation;
    a.opacity_offset = P->opacity_offset;
    if (f) {
      if (sc->storage != WSR_STORE_F32) return hipErrorInvalidValue;
      a.p_means = const_cast<float*>(static_cast<const float*>(sc->means));
      a.p_log_scales = const_cast<float*>(static_cast<const float*>(sc->log_scales));
      a.p_quats = const_cast<float*>(static_cast<const float*>(sc->quats));
      a.p_sh = const_cast<float*>(static_cast<const float*>(sc->sh));
      a.p_logit = const_cast<float*>(sc->opacity_logit);
      a.p_lc_v = const_cast<float*>(sc->lc_v);
      a.m = f->m;
      a.v = f->v;
      for (int k = 0; k < 7; ++k) a.lr[k] = f->lr[k];
      a.as = f->step;
      e = bwd_s<WSR_STORE_F32, true>(a, sc->sh_degree, blocks, st);
    } else {
      switch (sc->storage) {
        case WSR_STORE_F16: e = bwd_s<WSR_STORE_F16, false>(a, sc->sh_degree, blocks, st); break;
        case WSR_STORE_BF16: e = bwd_s<WSR_STORE_BF16, false>(a, sc->sh_degree, blocks, st); break;
        default: e = bwd_s<WSR_STORE_F32, false>(a, sc->sh_degree, blocks, st); break;
      }
    }
  } else {
    e = launch_fill_zero(gpart, 2 * sizeof(double), st);
  }
  if (e != hipSuccess) return e;
  reduce_globals<<<1, 1024, 0, st>>>(gpart, static_cast<int64_t>(blocks), at<float>(ws, L.off_tilepart),
                                    L.total_tiles, g->globals);
  return hipGetLastError();
}

hipError_t launch_project_bwd(const wsr_scene* sc, const wsr_params* P, const float* globals,
                              const Layout& L, void* ws, const void* pairs, int64_t capacity,
                              const wsr_grads* g, float* out_grad2d, hipStream_t st) {
  return project_bwd_impl(sc, P, globals, L, ws, pairs, capacity, g, nullptr, out_grad2d, st);
}

hipError_t launch_project_bwd_adam(const wsr_scene* sc, const wsr_params* P, const float* globals,
                                   const Layout& L, void* ws, const void* pairs, int64_t capacity,
                                   const FusedAdam& f, float* grad_globals, float* out_grad2d, hipStream_t st) {
  wsr_grads g = {};
  g.globals = grad_globals;
  return project_bwd_impl(sc, P, globals, L, ws, pairs, capacity, &g, &f, out_grad2d, st);
}

}  // namespace wsr
