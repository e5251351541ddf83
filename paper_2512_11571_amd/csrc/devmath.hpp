// Small FP32 vector / rotation helpers for the rollout kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace cem {

struct V3f {
  float x, y, z;
};
__device__ __forceinline__ V3f v3(float x, float y, float z) { return V3f{x, y, z}; }
__device__ __forceinline__ V3f operator+(V3f a, V3f b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3f operator-(V3f a, V3f b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3f operator-(V3f a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3f operator*(float s, V3f a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(V3f a, V3f b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3f cross(V3f a, V3f b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// sin and cos of x (radians), for the bounded angles of the rollout
// (|x| < 2^12): Cody and Waite's reduction x = k pi/2 + r with pi/2 split into
// three FP32 parts (the products k * part are exact for such k), then the
// Taylor polynomials of sin (to r^9) and cos (to r^10) on |r| <= pi/4, whose
// truncation error is below 2^-28, and the quadrant k mod 4.
__device__ __forceinline__ void sincos_rad(float x, float *s, float *c) {
  const float k = rintf(x * 0.636619746685028076f);
  float r = fmaf(-k, 1.57079637050628662f, x);
  r = fmaf(-k, -4.37113882867379300e-08f, r);
  r = fmaf(-k, -1.77635683940025046e-15f, r);
  const float r2 = r * r;
  const float ps = fmaf(r * r2, -1.0f / 6.0f + r2 * (1.0f / 120.0f + r2 * (-1.0f / 5040.0f + r2 * (1.0f / 362880.0f))), r);
  const float pc =
      fmaf(r2, -0.5f + r2 * (1.0f / 24.0f + r2 * (-1.0f / 720.0f + r2 * (1.0f / 40320.0f + r2 * (-1.0f / 3628800.0f)))),
           1.0f);
  const int q = (int)k & 3;
  *s = q == 0 ? ps : (q == 1 ? pc : (q == 2 ? -ps : -pc));
  *c = q == 0 ? pc : (q == 1 ? -ps : (q == 2 ? -pc : ps));
}

// Rotation matrix as three rows.
struct M3f {
  V3f r0, r1, r2;
};
__device__ __forceinline__ V3f mul(const M3f &R, V3f v) { return v3(dot(R.r0, v), dot(R.r1, v), dot(R.r2, v)); }
__device__ __forceinline__ V3f mulT(const M3f &R, V3f v) {
  return v3(R.r0.x * v.x + R.r1.x * v.y + R.r2.x * v.z, R.r0.y * v.x + R.r1.y * v.y + R.r2.y * v.z,
            R.r0.z * v.x + R.r1.z * v.y + R.r2.z * v.z);
}

// Unit quaternion (w, x, y, z), body -> world.
struct Q4f {
  float w, x, y, z;
};
__device__ __forceinline__ M3f rot_of(const Q4f &q) {
  const float xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
  const float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
  const float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
  M3f R;
  R.r0 = v3(1.0f - 2.0f * (yy + zz), 2.0f * (xy - wz), 2.0f * (xz + wy));
  R.r1 = v3(2.0f * (xy + wz), 1.0f - 2.0f * (xx + zz), 2.0f * (yz - wx));
  R.r2 = v3(2.0f * (xz - wy), 2.0f * (yz + wx), 1.0f - 2.0f * (xx + yy));
  return R;
}

}  // namespace cem
