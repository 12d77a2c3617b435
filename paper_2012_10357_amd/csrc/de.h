// Distance estimators of the seven primitive types, float32, local space.
//
// The paper names the procedural primitives of its sample scene -- CSG
// pac-men, a 3-D (quaternion) Julia set and a Mandelbulb, each behind an
// intersection shader (Sec. 4, listing "Hit group creation"; Figs. 1, 4-6)
// -- but leaves their device code to a separate chapter.  The definitions
// here are the textbook ones:
//   sphere      |p| - r
//   box         |max(q,0)| + min(max_i q_i, 0),  q = |p - c| - h
//   torus       |(sqrt(x^2+z^2) - R, y)| - r
//   box-frame   min over the 3 edge bars at the (+,+,+) corner of |p|
//               (mirror symmetry makes this the min over all 12 bars)
//   pac-man     max(|p| - R, -W(p)), W = signed distance to the wedge
//               |atan2(y, x)| <= alpha extruded along z
//   Julia       z <- z^2 + c over quaternions from (x, y, z, 0); derivative
//               m <- 2|z| m; stop when |z| > bailout; DE = |z| ln|z| / (2m)
//   Mandelbulb  power-8 spherical map (theta from +z, phi = atan2(y, x)),
//               dr <- 8 r^7 dr + 1; stop when r > bailout;
//               DE = ln(r) r / (2 dr) with r = |z| after the loop.
// Performance forms (same mathematics, different evaluation order):
//  - Julia carries |z|^2 and m^2, so its loop has no square root, and
//    DE = ln(|z|^2) sqrt(|z|^2 / m^2) / 4;
//  - the Mandelbulb map is evaluated without trigonometry:
//    (z + i rho)^8 = r^8 (cos 8th + i sin 8th) by three complex squarings
//    that keep the odd powers of rho factored out, and
//    ((x + i y) / rho)^8 = cos 8ph + i sin 8ph by three unit-complex
//    squarings; on the polar axis (rho = 0) phi is taken as 0.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/procray.h"

namespace pr {

// Hardware square root and base-2 logarithm (about 1 ulp) instead of the
// correctly rounded library expansions: the march only compares values with
// eps and accumulates them, so the last-bit rounding does not matter, while
// the expansions cost ~15 instructions each in the innermost loop.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fln(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }

// parameter slots after packing on the host
//   SPHERE     r
//   BOX        cx cy cz hx hy hz
//   TORUS      R r
//   BOXFRAME   b e (b - e)
//   PACMAN     R cos(alpha) sin(alpha)
//   JULIA      c0 c1 c2 c3 n_iter bailout^2
//   MANDELBULB n_iter bailout^2

__device__ __forceinline__ float box_q(float qx, float qy, float qz) {
  float ox = fmaxf(qx, 0.0f), oy = fmaxf(qy, 0.0f), oz = fmaxf(qz, 0.0f);
  float out = fsqrt(ox * ox + oy * oy + oz * oz);
  return out + fminf(fmaxf(qx, fmaxf(qy, qz)), 0.0f);
}

__device__ __forceinline__ float de_sphere(float x, float y, float z, const float* k) {
  return fsqrt(x * x + y * y + z * z) - k[0];
}

__device__ __forceinline__ float de_box(float x, float y, float z, const float* k) {
  return box_q(fabsf(x - k[0]) - k[3], fabsf(y - k[1]) - k[4], fabsf(z - k[2]) - k[5]);
}

__device__ __forceinline__ float de_torus(float x, float y, float z, const float* k) {
  float a = fsqrt(x * x + z * z) - k[0];
  return fsqrt(a * a + y * y) - k[1];
}

__device__ __forceinline__ float de_boxframe(float x, float y, float z, const float* k) {
  const float b = k[0], e = k[1], m = k[2];
  float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
  float dx = fabsf(ax - m) - e, dy = fabsf(ay - m) - e, dz = fabsf(az - m) - e;
  float bx = box_q(ax - b, dy, dz);
  float by = box_q(dx, ay - b, dz);
  float bz = box_q(dx, dy, az - b);
  return fminf(bx, fminf(by, bz));
}

__device__ __forceinline__ float de_pacman(float x, float y, float z, const float* k) {
  const float R = k[0], ca = k[1], sa = k[2];
  float len = fsqrt(x * x + y * y + z * z);
  float qx = x, qy = fabsf(y);
  float qn = -sa * qx + ca * qy;
  float qu = ca * qx + sa * qy;
  float w = (qn > 0.0f && qu < 0.0f) ? fsqrt(qx * qx + qy * qy) : qn;
  return fmaxf(len - R, -w);
}

// returns DE; *iters receives the number of map iterations executed
__device__ __forceinline__ float de_julia(float x, float y, float z, const float* k, int* iters) {
  const float c0 = k[0], c1 = k[1], c2 = k[2], c3 = k[3];
  const int nit = (int)k[4];
  const float bail2 = k[5];
  float zx = x, zy = y, zz = z, zw = 0.0f;
  float m2 = 1.0f;
  int it = 0;
  for (; it < nit; ++it) {
    float yzw = zy * zy + zz * zz + zw * zw;
    float r2 = zx * zx + yzw;
    if (r2 > bail2) break;
    m2 *= 4.0f * r2;
    float tx = zx + zx;
    float nx = zx * zx - yzw + c0;
    zy = tx * zy + c1;
    zz = tx * zz + c2;
    zw = tx * zw + c3;
    zx = nx;
  }
  *iters = it;
  float r2 = zx * zx + zy * zy + zz * zz + zw * zw;
  if (!(r2 > 1e-30f)) return 0.0f;
  return 0.25f * fln(r2) * fsqrt(r2 / m2);
}

__device__ __forceinline__ float de_mandelbulb(float px, float py, float pz, const float* k,
                                               int* iters) {
  const int nit = (int)k[0];
  const float bail2 = k[1];
  float x = px, y = py, z = pz, dr = 1.0f;
  int it = 0;
  for (; it < nit; ++it) {
    float rho2 = x * x + y * y;
    float r2 = rho2 + z * z;
    if (r2 > bail2) break;
    float r = fsqrt(r2);
    float r6 = r2 * r2 * r2;
    dr = 8.0f * r6 * r * dr + 1.0f;
    // (z + i rho)^8 = a3 + i rho b3
    float a1 = z * z - rho2, b1 = z + z;
    float a2 = a1 * a1 - rho2 * (b1 * b1), b2 = 2.0f * a1 * b1;
    float a3 = a2 * a2 - rho2 * (b2 * b2), b3 = 2.0f * a2 * b2;
    // ((x + i y) / rho)^8 = c8 + i s8
    float c = 1.0f, s = 0.0f, rho = 0.0f;
    if (rho2 > 1e-35f) {
      float ir = __builtin_amdgcn_rsqf(rho2);
      c = x * ir;
      s = y * ir;
      rho = rho2 * ir;
    }
    float c2 = c * c - s * s, s2 = 2.0f * c * s;
    float c4 = c2 * c2 - s2 * s2, s4 = 2.0f * c2 * s2;
    float c8 = c4 * c4 - s4 * s4, s8 = 2.0f * c4 * s4;
    float imA = rho * b3;
    x = imA * c8 + px;
    y = imA * s8 + py;
    z = a3 + pz;
  }
  *iters = it;
  float r = fsqrt(x * x + y * y + z * z);
  if (!(r > 1e-30f)) return 0.0f;
  return 0.5f * fln(r) * r / dr;
}

// ---------------------------------------------------------------------------
// Double-precision versions used only for the six central-difference taps of
// a normal.  Inside the fractals the float32 orbit of a non-escaping point is
// chaotic enough that a tap's value can be off by ~1e-5, which tilts the
// normal by about a percent; CDNA executes FP64 FMAs at the full rate of
// non-packed FP32, and taps are a small share of all evaluations.
__device__ __forceinline__ double box_q64(double qx, double qy, double qz) {
  double ox = fmax(qx, 0.0), oy = fmax(qy, 0.0), oz = fmax(qz, 0.0);
  return __builtin_sqrt(ox * ox + oy * oy + oz * oz) + fmin(fmax(qx, fmax(qy, qz)), 0.0);
}

__device__ __forceinline__ double de_eval64(uint32_t type, double x, double y, double z,
                                            const float* k, int* iters) {
  *iters = 0;
  switch (type) {
    case PR_SPHERE: return __builtin_sqrt(x * x + y * y + z * z) - (double)k[0];
    case PR_BOX:
      return box_q64(fabs(x - (double)k[0]) - (double)k[3], fabs(y - (double)k[1]) - (double)k[4],
                     fabs(z - (double)k[2]) - (double)k[5]);
    case PR_TORUS: {
      double a = __builtin_sqrt(x * x + z * z) - (double)k[0];
      return __builtin_sqrt(a * a + y * y) - (double)k[1];
    }
    case PR_BOXFRAME: {
      const double b = k[0], e = k[1], m = b - e;
      double ax = fabs(x), ay = fabs(y), az = fabs(z);
      double dx = fabs(ax - m) - e, dy = fabs(ay - m) - e, dz = fabs(az - m) - e;
      return fmin(box_q64(ax - b, dy, dz), fmin(box_q64(dx, ay - b, dz), box_q64(dx, dy, az - b)));
    }
    case PR_PACMAN: {
      const double R = k[0], ca = k[1], sa = k[2];
      double len = __builtin_sqrt(x * x + y * y + z * z);
      double qx = x, qy = fabs(y);
      double qn = -sa * qx + ca * qy, qu = ca * qx + sa * qy;
      double w = (qn > 0.0 && qu < 0.0) ? __builtin_sqrt(qx * qx + qy * qy) : qn;
      return fmax(len - R, -w);
    }
    case PR_JULIA: {
      const double c0 = k[0], c1 = k[1], c2 = k[2], c3 = k[3], bail2 = k[5];
      const int nit = (int)k[4];
      double zx = x, zy = y, zz = z, zw = 0.0, m2 = 1.0;
      int it = 0;
      for (; it < nit; ++it) {
        double yzw = zy * zy + zz * zz + zw * zw;
        double r2 = zx * zx + yzw;
        if (r2 > bail2) break;
        m2 *= 4.0 * r2;
        double tx = zx + zx;
        double nx = zx * zx - yzw + c0;
        zy = tx * zy + c1;
        zz = tx * zz + c2;
        zw = tx * zw + c3;
        zx = nx;
      }
      *iters = it;
      double r2 = zx * zx + zy * zy + zz * zz + zw * zw;
      if (!(r2 > 1e-300)) return 0.0;
      return 0.25 * log(r2) * __builtin_sqrt(r2 / m2);
    }
    default: {
      const int nit = (int)k[0];
      const double bail2 = k[1];
      double X = x, Y = y, Z = z, dr = 1.0;
      int it = 0;
      for (; it < nit; ++it) {
        double rho2 = X * X + Y * Y;
        double r2 = rho2 + Z * Z;
        if (r2 > bail2) break;
        double r = __builtin_sqrt(r2);
        dr = 8.0 * (r2 * r2 * r2) * r * dr + 1.0;
        double a1 = Z * Z - rho2, b1 = Z + Z;
        double a2 = a1 * a1 - rho2 * (b1 * b1), b2 = 2.0 * a1 * b1;
        double a3 = a2 * a2 - rho2 * (b2 * b2), b3 = 2.0 * a2 * b2;
        double c = 1.0, s = 0.0, rho = 0.0;
        if (rho2 > 1e-300) {
          rho = __builtin_sqrt(rho2);
          c = X / rho;
          s = Y / rho;
        }
        double c2 = c * c - s * s, s2 = 2.0 * c * s;
        double c4 = c2 * c2 - s2 * s2, s4 = 2.0 * c2 * s2;
        double c8 = c4 * c4 - s4 * s4, s8 = 2.0 * c4 * s4;
        double imA = rho * b3;
        X = imA * c8 + x;
        Y = imA * s8 + y;
        Z = a3 + z;
      }
      *iters = it;
      double r = __builtin_sqrt(X * X + Y * Y + Z * Z);
      if (!(r > 1e-300)) return 0.0;
      return 0.5 * log(r) * r / dr;
    }
  }
}

// Type switch: the kernel's replacement for the shader-table lookup of the
// paper's indexing rule (Sec. 2.2.3, Eq. 1): the instance record's type
// selects the intersection routine.
__device__ __forceinline__ float de_eval(uint32_t type, float x, float y, float z, const float* k,
                                         int* iters) {
  *iters = 0;
  switch (type) {
    case PR_SPHERE: return de_sphere(x, y, z, k);
    case PR_BOX: return de_box(x, y, z, k);
    case PR_TORUS: return de_torus(x, y, z, k);
    case PR_BOXFRAME: return de_boxframe(x, y, z, k);
    case PR_PACMAN: return de_pacman(x, y, z, k);
    case PR_JULIA: return de_julia(x, y, z, k, iters);
    default: return de_mandelbulb(x, y, z, k, iters);
  }
}

}  // namespace pr
