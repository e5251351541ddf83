// Oracle: rigid-body primitives, narrowphase and penalty contact.
// TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
//
// The state of the system is the robot configuration plus the SE(3) poses of
// the m objects (Sec. II, configuration space X = Q x SE(3)^m), advanced by
// the dynamics x_{t+1} = f(x_t, c_i, z_i) (Problem 1, Eq. 1b).  The paper runs
// a GPU physics engine for f; here f is written out: free rigid bodies under
// gravity, sphere/box/plane narrowphase, penalty normal forces with a damping
// term clamped at zero, regularised Coulomb friction, semi-implicit Euler.
#pragma once
#include "ref_scalar.hpp"

namespace ref {

template <class T> struct V3 {
  T x, y, z;
  V3() : x(0.0), y(0.0), z(0.0) {}
  V3(T a, T b, T c) : x(a), y(b), z(c) {}
};
template <class T> inline V3<T> operator+(const V3<T> &a, const V3<T> &b) { return V3<T>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class T> inline V3<T> operator-(const V3<T> &a, const V3<T> &b) { return V3<T>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class T> inline V3<T> operator-(const V3<T> &a) { return V3<T>(-a.x, -a.y, -a.z); }
template <class T> inline V3<T> operator*(T s, const V3<T> &a) { return V3<T>(s * a.x, s * a.y, s * a.z); }
template <class T> inline T dot(const V3<T> &a, const V3<T> &b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> inline V3<T> cross(const V3<T> &a, const V3<T> &b) {
  return V3<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class T> inline T norm(const V3<T> &a) { return r_sqrt(dot(a, a)); }

// Row-major 3x3.
template <class T> struct M3 { T m[3][3]; };
template <class T> inline V3<T> mul(const M3<T> &R, const V3<T> &v) {
  return V3<T>(R.m[0][0] * v.x + R.m[0][1] * v.y + R.m[0][2] * v.z,
               R.m[1][0] * v.x + R.m[1][1] * v.y + R.m[1][2] * v.z,
               R.m[2][0] * v.x + R.m[2][1] * v.y + R.m[2][2] * v.z);
}
template <class T> inline V3<T> mulT(const M3<T> &R, const V3<T> &v) {
  return V3<T>(R.m[0][0] * v.x + R.m[1][0] * v.y + R.m[2][0] * v.z,
               R.m[0][1] * v.x + R.m[1][1] * v.y + R.m[2][1] * v.z,
               R.m[0][2] * v.x + R.m[1][2] * v.y + R.m[2][2] * v.z);
}
template <class T> inline M3<T> matmul(const M3<T> &A, const M3<T> &B) {
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[i][0] * B.m[0][j] + A.m[i][1] * B.m[1][j] + A.m[i][2] * B.m[2][j];
  return C;
}
template <class T> inline M3<T> transpose(const M3<T> &A) {
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[j][i];
  return C;
}
template <class T> inline M3<T> eye3() {
  M3<T> I;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) I.m[i][j] = (i == j) ? T(1.0) : T(0.0);
  return I;
}
// Rotation about a principal axis (0 = x, 1 = y, 2 = z) by angle with cosine c, sine s.
template <class T> inline M3<T> axis_rot(int axis, T c, T s) {
  M3<T> R = eye3<T>();
  int a = (axis + 1) % 3, b = (axis + 2) % 3;
  R.m[a][a] = c; R.m[a][b] = -s;
  R.m[b][a] = s; R.m[b][b] = c;
  return R;
}

// Unit quaternion (w, x, y, z), Hamilton convention, body -> world.
template <class T> struct Q4 { T w, x, y, z; };
template <class T> inline M3<T> quat_to_mat(const Q4<T> &q) {
  M3<T> R;
  R.m[0][0] = T(1.0) - T(2.0) * (q.y * q.y + q.z * q.z);
  R.m[0][1] = T(2.0) * (q.x * q.y - q.w * q.z);
  R.m[0][2] = T(2.0) * (q.x * q.z + q.w * q.y);
  R.m[1][0] = T(2.0) * (q.x * q.y + q.w * q.z);
  R.m[1][1] = T(1.0) - T(2.0) * (q.x * q.x + q.z * q.z);
  R.m[1][2] = T(2.0) * (q.y * q.z - q.w * q.x);
  R.m[2][0] = T(2.0) * (q.x * q.z - q.w * q.y);
  R.m[2][1] = T(2.0) * (q.y * q.z + q.w * q.x);
  R.m[2][2] = T(1.0) - T(2.0) * (q.x * q.x + q.y * q.y);
  return R;
}

// A free rigid body: COM position, orientation, world linear and angular velocity.
template <class T> struct Body {
  V3<T> p;
  Q4<T> q;
  V3<T> v, w;
};

// Accumulated external wrench about the COM, world frame.
template <class T> struct Wrench {
  V3<T> f, tau;
};

// Semi-implicit Euler step of length h for a free body with mass m and
// principal (body-frame, diagonal) inertia Ib, under gravity vector gv:
//   v+ = v + h (F/m + gv)
//   w+ = w + h Iw^-1 (tau - w x Iw w),   Iw = R Ib R^T
//   p+ = p + h v+
//   q+ = normalize(q + (h/2) (0, w+) (x) q)
template <class T>
inline void integrate_free(Body<T> &b, const Wrench<T> &W, T m, const V3<T> &Ib, const V3<T> &gv, T h) {
  const M3<T> R = quat_to_mat(b.q);
  b.v = b.v + h * ((T(1.0) / m) * W.f + gv);
  const V3<T> wb = mulT(R, b.w);                     // body-frame angular velocity
  const V3<T> Lb(Ib.x * wb.x, Ib.y * wb.y, Ib.z * wb.z);
  const V3<T> gyro = mul(R, Lb);                     // Iw w in world
  const V3<T> rhs = W.tau - cross(b.w, gyro);
  const V3<T> rb = mulT(R, rhs);
  const V3<T> dwb(rb.x / Ib.x, rb.y / Ib.y, rb.z / Ib.z);
  b.w = b.w + h * mul(R, dwb);
  b.p = b.p + h * b.v;
  const T hh = T(0.5) * h;
  const Q4<T> q = b.q;
  Q4<T> dq;
  dq.w = -(b.w.x * q.x + b.w.y * q.y + b.w.z * q.z);
  dq.x = q.w * b.w.x + (b.w.y * q.z - b.w.z * q.y);
  dq.y = q.w * b.w.y + (b.w.z * q.x - b.w.x * q.z);
  dq.z = q.w * b.w.z + (b.w.x * q.y - b.w.y * q.x);
  Q4<T> qn;
  qn.w = q.w + hh * dq.w;
  qn.x = q.x + hh * dq.x;
  qn.y = q.y + hh * dq.y;
  qn.z = q.z + hh * dq.z;
  const T inv = T(1.0) / r_sqrt(qn.w * qn.w + qn.x * qn.x + qn.y * qn.y + qn.z * qn.z);
  b.q.w = qn.w * inv; b.q.x = qn.x * inv; b.q.y = qn.y * inv; b.q.z = qn.z * inv;
}

// One contact: point x (world), unit normal n pointing from B into A, depth d > 0.
template <class T> struct Contact {
  V3<T> x, n;
  T d;
};

// Penalty contact force on A at a contact, given the two material-point
// velocities at x:
//   f_n = max(0, k d - c v_n),  v_n = n . (vA - vB)
//   f_t = -mu f_n v_t / sqrt(|v_t|^2 + eps_v^2),  v_t = v_rel - v_n n
// Returns the force on A (B receives the negative).
template <class T>
inline V3<T> penalty_force(const Contact<T> &c, const V3<T> &vA, const V3<T> &vB, T k, T damp, T mu, T eps_v) {
  const V3<T> vr = vA - vB;
  const T vn = dot(c.n, vr);
  const T fn = r_max(T(0.0), k * c.d - damp * vn);
  const V3<T> vt = vr - vn * c.n;
  const T denom = r_sqrt(dot(vt, vt) + eps_v * eps_v);
  const T s = -(mu * fn) / denom;
  return fn * c.n + s * vt;
}

// Add a force F applied at world point x to a body's wrench about its COM p.
template <class T> inline void add_force(Wrench<T> &W, const V3<T> &p, const V3<T> &x, const V3<T> &F) {
  W.f = W.f + F;
  W.tau = W.tau + cross(x - p, F);
}

// Box (center p, rotation R, half extents he) against the plane z = 0:
// each of the 8 vertices below the plane is a contact with n = +z (A = box).
template <class T>
inline int box_plane(const V3<T> &p, const M3<T> &R, const V3<T> &he, Contact<T> out[8]) {
  int n = 0;
  for (int i = 0; i < 8; ++i) {
    const T sx = (i & 1) ? T(1.0) : T(-1.0);
    const T sy = (i & 2) ? T(1.0) : T(-1.0);
    const T sz = (i & 4) ? T(1.0) : T(-1.0);
    const V3<T> x = p + mul(R, V3<T>(sx * he.x, sy * he.y, sz * he.z));
    const T d = -x.z;
    if (d > T(0.0)) {
      out[n].x = x;
      out[n].n = V3<T>(T(0.0), T(0.0), T(1.0));
      out[n].d = d;
      ++n;
    }
  }
  return n;
}

// Index of the nearest face of a box (half extents he) to a point pb inside it,
// in the order +x, -x, +y, -y, +z, -z, lowest index on ties; dist gets the
// distance to that face.
template <class T> inline int nearest_face(const V3<T> &pb, const V3<T> &he, T *dist) {
  T ds[6] = {he.x - pb.x, he.x + pb.x, he.y - pb.y, he.y + pb.y, he.z - pb.z, he.z + pb.z};
  int best = 0;
  for (int f = 1; f < 6; ++f)
    if (ds[f] < ds[best]) best = f;
  *dist = ds[best];
  return best;
}
template <class T> inline V3<T> face_normal(int f) {
  const T s = (f & 1) ? T(-1.0) : T(1.0);
  if (f < 2) return V3<T>(s, T(0.0), T(0.0));
  if (f < 4) return V3<T>(T(0.0), s, T(0.0));
  return V3<T>(T(0.0), T(0.0), s);
}

// Sphere (center c, radius r) = B against box (p, R, he) = A.  Closest point of
// the box to the centre by clamping in the box frame; if the centre lies inside,
// the nearest face.  n points from the sphere into the box.  Returns 0 or 1.
template <class T>
inline int sphere_box(const V3<T> &c, T r, const V3<T> &p, const M3<T> &R, const V3<T> &he, Contact<T> *out) {
  const V3<T> cb = mulT(R, c - p);
  const V3<T> cp(r_max(-he.x, r_min(he.x, cb.x)), r_max(-he.y, r_min(he.y, cb.y)), r_max(-he.z, r_min(he.z, cb.z)));
  const V3<T> diff = cb - cp;
  const T d2 = dot(diff, diff);
  if (d2 > T(0.0)) {
    const T dist = r_sqrt(d2);
    const T depth = r - dist;
    if (!(depth > T(0.0))) return 0;
    const T inv = T(1.0) / dist;
    out->n = mul(R, -(inv * diff));
    out->x = p + mul(R, cp);
    out->d = depth;
    return 1;
  }
  T fd;
  const int f = nearest_face(cb, he, &fd);
  const V3<T> nf = face_normal<T>(f);
  V3<T> xb = cb;
  if (f < 2) xb.x = nf.x * he.x;
  else if (f < 4) xb.y = nf.y * he.y;
  else xb.z = nf.z * he.z;
  out->n = mul(R, -nf);
  out->x = p + mul(R, xb);
  out->d = r + fd;
  return 1;
}

// Broadphase for two boxes (centre p, rotation R box -> world, half extents h):
// the separating-axis test restricted to the six face normals.  Along the unit
// axis a, box A covers p_A.a +- sum_k h_A,k |a . R_A e_k|, and likewise B; if
// the two intervals are disjoint along one of these axes the boxes do not
// intersect, so no vertex of either lies inside the other.  It only skips
// vertex tests that find nothing; g_face_cull = false switches it off (every
// pair then runs the vertex tests), which the pins use to show that the
// rollouts do not change.
inline bool g_face_cull = true;
template <class T>
inline bool face_separated(const V3<T> &pA, const M3<T> &RA, const V3<T> &hA, const V3<T> &pB, const M3<T> &RB,
                           const V3<T> &hB) {
  if (!g_face_cull) return false;
  const V3<T> d = pB - pA;
  const T ha[3] = {hA.x, hA.y, hA.z}, hb[3] = {hB.x, hB.y, hB.z};
  for (int side = 0; side < 2; ++side) {
    const M3<T> &R1 = side == 0 ? RA : RB, &R2 = side == 0 ? RB : RA;
    const T *h1 = side == 0 ? ha : hb, *h2 = side == 0 ? hb : ha;
    for (int k = 0; k < 3; ++k) {
      const V3<T> a(R1.m[0][k], R1.m[1][k], R1.m[2][k]);
      T r2 = T(0.0);
      for (int j = 0; j < 3; ++j) r2 = r2 + h2[j] * r_abs(dot(a, V3<T>(R2.m[0][j], R2.m[1][j], R2.m[2][j])));
      if (r_abs(dot(a, d)) > h1[k] + r2) return true;
    }
  }
  return false;
}

// Vertex-face test of box A's vertices against box B (both dynamic or B static):
// every vertex of A strictly inside B is a contact with depth = distance to
// B's nearest face and n = that face's outward normal (from B into A).
template <class T>
inline int box_verts_in_box(const V3<T> &pA, const M3<T> &RA, const V3<T> &heA, const V3<T> &pB,
                            const M3<T> &RB, const V3<T> &heB, Contact<T> out[8]) {
  int n = 0;
  for (int i = 0; i < 8; ++i) {
    const T sx = (i & 1) ? T(1.0) : T(-1.0);
    const T sy = (i & 2) ? T(1.0) : T(-1.0);
    const T sz = (i & 4) ? T(1.0) : T(-1.0);
    const V3<T> x = pA + mul(RA, V3<T>(sx * heA.x, sy * heA.y, sz * heA.z));
    const V3<T> xb = mulT(RB, x - pB);
    if (r_abs(xb.x) < heB.x && r_abs(xb.y) < heB.y && r_abs(xb.z) < heB.z) {
      T fd;
      const int f = nearest_face(xb, heB, &fd);
      out[n].x = x;
      out[n].n = mul(RB, face_normal<T>(f));
      out[n].d = fd;
      ++n;
    }
  }
  return n;
}

}  // namespace ref
