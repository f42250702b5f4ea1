// Per-(view, Gaussian) geometry shared by the projection and its backward,
// so both take the same visibility decisions: view transform, near-plane
// cull, EWA projection Sigma2D = (J W) Sigma3D (J W)^T + dilation (Sec. 3,
// Eq. 5), its inverse (the conic) and the projected centre.  Double
// precision throughout (the centre must be exact to ~1e-9 px of its value).
#pragma once

#include "wsr_internal.h"

namespace wsr {

struct Sigma3 {
  double s[6];  // xx, xy, xz, yy, yz, zz
};

struct QuatScale {
  double w, x, y, z;  // unit quaternion
  double s0, s1, s2;  // scales
  double R[9];        // rotation, row-major
  bool ok;
};

// Normalise the quaternion (a zero quaternion has no rotation: not ok) and
// build R(q) and Sigma3D = R diag(s^2) R^T.
__device__ inline Sigma3 make_sigma3(double qw, double qx, double qy, double qz, double ls0, double ls1,
                                     double ls2, QuatScale* qs) {
  const double n2 = qw * qw + qx * qx + qy * qy + qz * qz;
  qs->ok = n2 > 0.0;
  const double inv = qs->ok ? 1.0 / sqrt(n2) : 0.0;
  const double w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  qs->w = w; qs->x = x; qs->y = y; qs->z = z;
  qs->s0 = exp(ls0); qs->s1 = exp(ls1); qs->s2 = exp(ls2);
  double* R = qs->R;
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
  const double s[3] = {qs->s0 * qs->s0, qs->s1 * qs->s1, qs->s2 * qs->s2};
  Sigma3 S;
  S.s[0] = R[0] * R[0] * s[0] + R[1] * R[1] * s[1] + R[2] * R[2] * s[2];
  S.s[1] = R[0] * R[3] * s[0] + R[1] * R[4] * s[1] + R[2] * R[5] * s[2];
  S.s[2] = R[0] * R[6] * s[0] + R[1] * R[7] * s[1] + R[2] * R[8] * s[2];
  S.s[3] = R[3] * R[3] * s[0] + R[4] * R[4] * s[1] + R[5] * R[5] * s[2];
  S.s[4] = R[3] * R[6] * s[0] + R[4] * R[7] * s[1] + R[5] * R[8] * s[2];
  S.s[5] = R[6] * R[6] * s[0] + R[7] * R[7] * s[1] + R[8] * R[8] * s[2];
  return S;
}

struct ViewGeom {
  double W[9];            // camera rotation
  double tx, ty, tz, izt;
  double rx, ry;          // lateral ratios after the clamp
  bool unclamped_x, unclamped_y;
  double a[3], b[3];      // rows of J W
  double c00, c01, c11;   // Sigma2D including the dilation
  double A, B, C;         // conic
  double mux, muy;        // projected centre (pixels)
};

__device__ inline void sym_mul(const Sigma3& S, const double v[3], double o[3]) {
  o[0] = S.s[0] * v[0] + S.s[1] * v[1] + S.s[2] * v[2];
  o[1] = S.s[1] * v[0] + S.s[3] * v[1] + S.s[4] * v[2];
  o[2] = S.s[2] * v[0] + S.s[4] * v[1] + S.s[5] * v[2];
}

// Returns true iff the pair is visible (in front of the near plane, positive
// definite Sigma2D, centre within +-2^22 px so that pixel offsets from its integer
// origin are exact half-integers in float32).
__device__ inline bool view_geom(const DevCamera& cam, double p0, double p1, double p2, const Sigma3& S,
                                 bool q_ok, float near_z, float dilation, ViewGeom* g) {
#pragma unroll
  for (int k = 0; k < 9; ++k) g->W[k] = cam.R[k];
  const double* W = g->W;
  g->tx = W[0] * p0 + W[1] * p1 + W[2] * p2 + cam.T[0];
  g->ty = W[3] * p0 + W[4] * p1 + W[5] * p2 + cam.T[1];
  g->tz = W[6] * p0 + W[7] * p1 + W[8] * p2 + cam.T[2];
  if (!q_ok || !(g->tz > static_cast<double>(near_z))) return false;
  const double fx = cam.fx, fy = cam.fy;
  g->izt = 1.0 / g->tz;
  const double limx = 1.3 * 0.5 * cam.width / fx, limy = 1.3 * 0.5 * cam.height / fy;
  const double ux = g->tx * g->izt, uy = g->ty * g->izt;
  g->unclamped_x = ux >= -limx && ux <= limx;
  g->unclamped_y = uy >= -limy && uy <= limy;
  g->rx = fmin(fmax(ux, -limx), limx);
  g->ry = fmin(fmax(uy, -limy), limy);
  const double kx = fx * g->izt, ky = fy * g->izt;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    g->a[j] = kx * (W[j] - g->rx * W[6 + j]);
    g->b[j] = ky * (W[3 + j] - g->ry * W[6 + j]);
  }
  double Sa[3], Sb[3];
  sym_mul(S, g->a, Sa);
  sym_mul(S, g->b, Sb);
  g->c00 = g->a[0] * Sa[0] + g->a[1] * Sa[1] + g->a[2] * Sa[2] + dilation;
  g->c01 = g->b[0] * Sa[0] + g->b[1] * Sa[1] + g->b[2] * Sa[2];
  g->c11 = g->b[0] * Sb[0] + g->b[1] * Sb[1] + g->b[2] * Sb[2] + dilation;
  const double det = g->c00 * g->c11 - g->c01 * g->c01;
  if (!(det > 0.0)) return false;
  const double id = 1.0 / det;
  g->A = g->c11 * id;
  g->B = -g->c01 * id;
  g->C = g->c00 * id;
  g->mux = fx * g->tx * g->izt + cam.cx;
  g->muy = fy * g->ty * g->izt + cam.cy;
  return fabs(g->mux) < 4194304.0 && fabs(g->muy) < 4194304.0;
}

// Unit direction from the camera centre (-W^T T) to p, W the camera
// rotation (as view_geom reads it from the camera).
__device__ inline void view_dir_w(const double* W, const DevCamera& cam, double p0, double p1, double p2,
                                  double d[3], double* len) {
  const double fx = -(W[0] * cam.T[0] + W[3] * cam.T[1] + W[6] * cam.T[2]);
  const double fy = -(W[1] * cam.T[0] + W[4] * cam.T[1] + W[7] * cam.T[2]);
  const double fz = -(W[2] * cam.T[0] + W[5] * cam.T[1] + W[8] * cam.T[2]);
  const double vx = p0 - fx, vy = p1 - fy, vz = p2 - fz;
  *len = sqrt(vx * vx + vy * vy + vz * vz);
  const double il = 1.0 / *len;
  d[0] = vx * il;
  d[1] = vy * il;
  d[2] = vz * il;
}

__device__ inline void view_dir(const ViewGeom& g, const DevCamera& cam, double p0, double p1, double p2,
                                double d[3], double* len) {
  view_dir_w(g.W, cam, p0, p1, p2, d, len);
}

// The same direction straight from the camera, before (or without) view_geom.
__device__ inline void view_dir_cam(const DevCamera& cam, double p0, double p1, double p2, double d[3],
                                    double* len) {
  double W[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) W[k] = cam.R[k];
  view_dir_w(W, cam, p0, p1, p2, d, len);
}

}  // namespace wsr
