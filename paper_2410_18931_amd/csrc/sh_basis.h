// Real orthonormal spherical harmonics, degrees 0-3, on a unit direction
// (x, y, z); coefficient index k = l*l + l + m.  Each basis function is the
// homogeneous harmonic polynomial of degree l scaled to unit L2 norm on the
// sphere (m > 0: cos(m phi) family, m < 0: sin(|m| phi) family).
//
// sh_eval_grad returns the gradient of each polynomial with respect to the
// three components; only its tangential part matters, because callers chain
// it through the Jacobian of the normalisation dir = v / |v|.
#pragma once

namespace wsr {

// Normalisation constants.
constexpr float kY00 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kY1 = 0.48860251190291992f;    // sqrt(3 / (4 pi))
constexpr float kY2a = 1.0925484305920792f;    // sqrt(15 / pi) / 2
constexpr float kY2b = 0.31539156525252005f;   // sqrt(5 / pi) / 4
constexpr float kY2c = 0.54627421529603959f;   // sqrt(15 / pi) / 4
constexpr float kY3a = 0.59004358992664352f;   // sqrt(35 / (2 pi)) / 4
constexpr float kY3b = 2.8906114426405538f;    // sqrt(105 / pi) / 2
constexpr float kY3c = 0.45704579946446572f;   // sqrt(21 / (2 pi)) / 4
constexpr float kY3d = 0.37317633259011540f;   // sqrt(7 / pi) / 4
constexpr float kY3e = 1.4453057213202769f;    // sqrt(105 / pi) / 4

template <int DEG>
__device__ inline void sh_eval(float x, float y, float z, float* Y) {
  Y[0] = kY00;
  if constexpr (DEG >= 1) {
    Y[1] = kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = kY1 * x;
  }
  if constexpr (DEG >= 2) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = kY2a * y * z;
    Y[6] = kY2b * (2.f * z2 - x2 - y2);
    Y[7] = kY2a * x * z;
    Y[8] = kY2c * (x2 - y2);
    if constexpr (DEG >= 3) {
      Y[9] = kY3a * y * (3.f * x2 - y2);
      Y[10] = kY3b * x * y * z;
      Y[11] = kY3c * y * (4.f * z2 - x2 - y2);
      Y[12] = kY3d * z * (2.f * z2 - 3.f * x2 - 3.f * y2);
      Y[13] = kY3c * x * (4.f * z2 - x2 - y2);
      Y[14] = kY3e * z * (x2 - y2);
      Y[15] = kY3a * x * (x2 - 3.f * y2);
    }
  }
}

// The same basis in double precision, for the opacity early-out's cutoff
// (a support decision, where a float32 opacity would move the cutoff by
// more than float rounding of q).
template <int DEG>
__device__ inline void sh_eval_f64(double x, double y, double z, double* Y) {
  Y[0] = 0.28209479177387814;
  if constexpr (DEG >= 1) {
    const double c1 = 0.48860251190291992;
    Y[1] = c1 * y;
    Y[2] = c1 * z;
    Y[3] = c1 * x;
  }
  if constexpr (DEG >= 2) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double a = 1.0925484305920792, b = 0.31539156525252005, c = 0.54627421529603959;
    Y[4] = a * x * y;
    Y[5] = a * y * z;
    Y[6] = b * (2.0 * z2 - x2 - y2);
    Y[7] = a * x * z;
    Y[8] = c * (x2 - y2);
    if constexpr (DEG >= 3) {
      const double e = 0.59004358992664352, f = 2.8906114426405538, g = 0.45704579946446572,
                   h = 0.37317633259011540, k = 1.4453057213202769;
      Y[9] = e * y * (3.0 * x2 - y2);
      Y[10] = f * x * y * z;
      Y[11] = g * y * (4.0 * z2 - x2 - y2);
      Y[12] = h * z * (2.0 * z2 - 3.0 * x2 - 3.0 * y2);
      Y[13] = g * x * (4.0 * z2 - x2 - y2);
      Y[14] = k * z * (x2 - y2);
      Y[15] = e * x * (x2 - 3.0 * y2);
    }
  }
}

// G[k] = (dY_k/dx, dY_k/dy, dY_k/dz) of the polynomials above.
template <int DEG>
__device__ inline void sh_eval_grad(float x, float y, float z, float3* G) {
  G[0] = make_float3(0.f, 0.f, 0.f);
  if constexpr (DEG >= 1) {
    G[1] = make_float3(0.f, kY1, 0.f);
    G[2] = make_float3(0.f, 0.f, kY1);
    G[3] = make_float3(kY1, 0.f, 0.f);
  }
  if constexpr (DEG >= 2) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    G[4] = make_float3(kY2a * y, kY2a * x, 0.f);
    G[5] = make_float3(0.f, kY2a * z, kY2a * y);
    G[6] = make_float3(-2.f * kY2b * x, -2.f * kY2b * y, 4.f * kY2b * z);
    G[7] = make_float3(kY2a * z, 0.f, kY2a * x);
    G[8] = make_float3(2.f * kY2c * x, -2.f * kY2c * y, 0.f);
    if constexpr (DEG >= 3) {
      G[9] = make_float3(6.f * kY3a * x * y, 3.f * kY3a * (x2 - y2), 0.f);
      G[10] = make_float3(kY3b * y * z, kY3b * x * z, kY3b * x * y);
      G[11] = make_float3(-2.f * kY3c * x * y, kY3c * (4.f * z2 - x2 - 3.f * y2), 8.f * kY3c * y * z);
      G[12] = make_float3(-6.f * kY3d * x * z, -6.f * kY3d * y * z, kY3d * (6.f * z2 - 3.f * x2 - 3.f * y2));
      G[13] = make_float3(kY3c * (4.f * z2 - 3.f * x2 - y2), -2.f * kY3c * x * y, 8.f * kY3c * x * z);
      G[14] = make_float3(2.f * kY3e * x * z, -2.f * kY3e * y * z, kY3e * (x2 - y2));
      G[15] = make_float3(3.f * kY3a * (x2 - y2), -6.f * kY3a * x * y, 0.f);
    }
  }
}

}  // namespace wsr
