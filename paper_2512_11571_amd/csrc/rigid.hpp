// Free rigid bodies, narrowphase and penalty contact for the rollout kernels
// (the dynamics f of Problem 1, Eq. 1b, written out for the GPU).
//
//  - contact: point x, normal n from B into A, depth d > 0;
//    f_n = max(0, k d - c v_n), f_t = -mu f_n v_t / sqrt(|v_t|^2 + eps_v^2)
//  - semi-implicit Euler: v, w first (gyroscopic term explicit, world-frame w),
//    then p and the quaternion (first order, renormalised).
// Contact loops test every candidate, then form forces in one pass per
// contact of a lane (a wave runs as many passes as its busiest lane).
#pragma once
#include "devmath.hpp"

namespace cem {

struct FreeBody {
  V3f p;
  Q4f q;
  V3f v, w;
};

struct Wrench {
  V3f f, t;
};

// Penalty force on A; `on` masks inactive contacts (returns exactly zero).
// The regularised friction's 1 / sqrt(|v_t|^2 + eps_v^2) is the hardware's
// reciprocal square root (about 1 ulp; its argument is at least eps_v^2 > 0).
__device__ __forceinline__ V3f contact_force(bool on, V3f n, float d, V3f vrel, float k, float damp, float mu,
                                             float eps2) {
  const float vn = dot(n, vrel);
  const float fn = on ? fmaxf(0.0f, k * d - damp * vn) : 0.0f;
  const V3f vt = vrel - vn * n;
  const float s = -(mu * fn) * __builtin_amdgcn_rsqf(dot(vt, vt) + eps2);
  return fn * n + s * vt;
}

// The same force in the frame of box B, whose face normal there is sgn e_ax:
// the normal speed is one component of vrel, the tangential velocity is vrel
// with that component zero, and the force's component ax is the normal force.
__device__ __forceinline__ V3f contact_force_b(int ax, float sgn, float d, V3f vrel, float k, float damp, float mu,
                                               float eps2) {
  const float va = ax == 0 ? vrel.x : (ax == 1 ? vrel.y : vrel.z);
  const float fn = fmaxf(0.0f, k * d - damp * (sgn * va));
  const V3f vt = v3(ax == 0 ? 0.0f : vrel.x, ax == 1 ? 0.0f : vrel.y, ax == 2 ? 0.0f : vrel.z);
  const float s = -(mu * fn) * __builtin_amdgcn_rsqf(dot(vt, vt) + eps2);  // as in contact_force
  const float f = fn * sgn;
  return v3(ax == 0 ? f : s * vt.x, ax == 1 ? f : s * vt.y, ax == 2 ? f : s * vt.z);
}

__device__ __forceinline__ void apply(Wrench &W, V3f r, V3f F) {
  W.f = W.f + F;
  W.t = W.t + cross(r, F);
}

// Box corners against the plane z = 0 (A = box, B = ground at rest).  The
// corner heights come from the third row of R alone; the lever arm and the
// force are formed once per corner below the plane of a lane, in ascending
// corner order, so lanes whose corners below the plane differ share passes.
// Only the corners in `vmask` (bit i: corner i) are taken.
__device__ __forceinline__ void box_ground(const FreeBody &b, const M3f &R, V3f he, float k, float damp, float mu,
                                           float eps2, Wrench &W, unsigned vmask = 0xFFu) {
  const float zx = he.x * R.r2.x, zy = he.y * R.r2.y, zz = he.z * R.r2.z;
  unsigned below = 0u;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float rz = ((i & 4) ? zz : -zz) + ((i & 2) ? zy : -zy) + ((i & 1) ? zx : -zx);
    if (-(b.p.z + rz) > 0.0f) below |= 1u << i;
  }
  below &= vmask;
  while (below != 0u) {  // at most eight passes
    const int i = __builtin_ctz(below);
    below &= below - 1u;
    const float rz = ((i & 4) ? zz : -zz) + ((i & 2) ? zy : -zy) + ((i & 1) ? zx : -zx);
    const float d = -(b.p.z + rz);
    const V3f loc = v3((i & 1) ? he.x : -he.x, (i & 2) ? he.y : -he.y, (i & 4) ? he.z : -he.z);
    const V3f r = mul(R, loc);
    const V3f vA = b.v + cross(b.w, r);
    apply(W, r, contact_force(true, v3(0.0f, 0.0f, 1.0f), d, vA, k, damp, mu, eps2));
  }
}

// Sphere B (centre c, radius rad, velocity vB) against box A: closest point
// by clamping in the box frame, nearest face when the centre is inside.
__device__ __forceinline__ void sphere_on_box(const FreeBody &b, const M3f &R, V3f he, V3f c, float rad, V3f vB,
                                              float k, float damp, float mu, float eps2, Wrench &W) {
  const V3f cb = mulT(R, c - b.p);
  const V3f cp = v3(fminf(fmaxf(cb.x, -he.x), he.x), fminf(fmaxf(cb.y, -he.y), he.y), fminf(fmaxf(cb.z, -he.z), he.z));
  const V3f diff = cb - cp;
  const float d2 = dot(diff, diff);
  V3f nb, xb;
  float depth;
  if (d2 > 0.0f) {
    const float dist = sqrtf(d2);
    depth = rad - dist;
    nb = (-1.0f / dist) * diff;
    xb = cp;
  } else {
    // nearest face, order +x -x +y -y +z -z, first on ties
    const float ds[6] = {he.x - cb.x, he.x + cb.x, he.y - cb.y, he.y + cb.y, he.z - cb.z, he.z + cb.z};
    int f = 0;
    float dmin = ds[0];
#pragma unroll
    for (int j = 1; j < 6; ++j) {
      const bool lt = ds[j] < dmin;
      f = lt ? j : f;
      dmin = lt ? ds[j] : dmin;
    }
    const float sgn = (f & 1) ? -1.0f : 1.0f;
    const int ax = f >> 1;
    nb = v3(ax == 0 ? -sgn : 0.0f, ax == 1 ? -sgn : 0.0f, ax == 2 ? -sgn : 0.0f);
    xb = v3(ax == 0 ? sgn * he.x : cb.x, ax == 1 ? sgn * he.y : cb.y, ax == 2 ? sgn * he.z : cb.z);
    depth = rad + dmin;
  }
  const V3f r = mul(R, xb);
  const V3f n = mul(R, nb);
  const V3f vA = b.v + cross(b.w, r);
  const V3f F = contact_force(depth > 0.0f, n, depth, vA - vB, k, damp, mu, eps2);
  apply(W, r, F);
}

// Semi-implicit Euler step with principal inertia Ib (body frame; inv_Ib its
// reciprocals), gravity gv and R = rot_of(b.q).  The quaternion's
// renormalisation takes the hardware's reciprocal square root (about 1 ulp).
__device__ __forceinline__ void integrate(FreeBody &b, const Wrench &W, float inv_m, V3f Ib, V3f inv_Ib, V3f gv,
                                          float h, const M3f &R) {
  b.v = b.v + h * (inv_m * W.f + gv);
  const V3f wb = mulT(R, b.w);
  const V3f Lw = mul(R, v3(Ib.x * wb.x, Ib.y * wb.y, Ib.z * wb.z));
  const V3f rb = mulT(R, W.t - cross(b.w, Lw));
  b.w = b.w + h * mul(R, v3(rb.x * inv_Ib.x, rb.y * inv_Ib.y, rb.z * inv_Ib.z));
  b.p = b.p + h * b.v;
  const float hh = 0.5f * h;
  const Q4f q = b.q;
  const V3f w = b.w;
  const float nw = q.w - hh * (w.x * q.x + w.y * q.y + w.z * q.z);
  const float nx = q.x + hh * (q.w * w.x + w.y * q.z - w.z * q.y);
  const float ny = q.y + hh * (q.w * w.y + w.z * q.x - w.x * q.z);
  const float nz = q.z + hh * (q.w * w.z + w.x * q.y - w.y * q.x);
  const float inv = __builtin_amdgcn_rsqf(nw * nw + nx * nx + ny * ny + nz * nz);
  b.q = Q4f{nw * inv, nx * inv, ny * inv, nz * inv};
}

}  // namespace cem
