// Spatial algebra, kinematics, IK and contact helpers of the mobile-manipulator rollout.
#pragma once
#include "internal.hpp"
#include "rigid.hpp"

namespace cem {
namespace {

constexpr int NJ = 11, ARM0 = 3, NARM = 6, FL = 9, FR = 10, BASEB = 2, PALM = 8;

// ---- spatial algebra (motion [w; v], force [n; f], body coordinates) ----
struct SV {
  V3f a, b;  // angular / linear part (motion) or moment / force part (force)
};
__device__ __forceinline__ SV sv(V3f a, V3f b) { return SV{a, b}; }
__device__ __forceinline__ SV operator+(SV x, SV y) { return sv(x.a + y.a, x.b + y.b); }
__device__ __forceinline__ SV operator-(SV x, SV y) { return sv(x.a - y.a, x.b - y.b); }
__device__ __forceinline__ SV operator*(float s, SV x) { return sv(s * x.a, s * x.b); }
__device__ __forceinline__ float dot6(SV x, SV y) { return dot(x.a, y.a) + dot(x.b, y.b); }
// v x m (motion) and v x* f (force)
__device__ __forceinline__ SV crm(SV v, SV m) { return sv(cross(v.a, m.a), cross(v.a, m.b) + cross(v.b, m.a)); }
__device__ __forceinline__ SV crf(SV v, SV f) { return sv(cross(v.a, f.a) + cross(v.b, f.b), cross(v.a, f.b)); }

// Symmetric 6x6 [A B; B^T C], A and C symmetric (xx xy xz yy yz zz), B row-major.
struct Sym6 {
  float A[6], B[9], C[6];
};
__device__ __forceinline__ V3f symv(const float *S, V3f x) {
  return v3(S[0] * x.x + S[1] * x.y + S[2] * x.z, S[1] * x.x + S[3] * x.y + S[4] * x.z,
            S[2] * x.x + S[4] * x.y + S[5] * x.z);
}
__device__ __forceinline__ V3f matv(const float *B, V3f x) {
  return v3(B[0] * x.x + B[1] * x.y + B[2] * x.z, B[3] * x.x + B[4] * x.y + B[5] * x.z,
            B[6] * x.x + B[7] * x.y + B[8] * x.z);
}
__device__ __forceinline__ V3f matTv(const float *B, V3f x) {
  return v3(B[0] * x.x + B[3] * x.y + B[6] * x.z, B[1] * x.x + B[4] * x.y + B[7] * x.z,
            B[2] * x.x + B[5] * x.y + B[8] * x.z);
}
__device__ __forceinline__ SV sym_mul(const Sym6 &I, SV m) {
  return sv(symv(I.A, m.a) + matv(I.B, m.b), matTv(I.B, m.a) + symv(I.C, m.b));
}
// column k (0..5) of I: k < 3 -> [A e_k; B^T e_k] (B^T e_k = row k of B);
// k >= 3 -> [B e_j; C e_j] (B e_j = column j of B), j = k - 3.  k is the same
// for the whole wave; each case reads fixed elements, so I stays in registers.
__device__ __forceinline__ SV sym_col(const Sym6 &I, int k) {
  SV o;
  switch (k) {
    case 0: o = sv(v3(I.A[0], I.A[1], I.A[2]), v3(I.B[0], I.B[1], I.B[2])); break;
    case 1: o = sv(v3(I.A[1], I.A[3], I.A[4]), v3(I.B[3], I.B[4], I.B[5])); break;
    case 2: o = sv(v3(I.A[2], I.A[4], I.A[5]), v3(I.B[6], I.B[7], I.B[8])); break;
    case 3: o = sv(v3(I.B[0], I.B[3], I.B[6]), v3(I.C[0], I.C[1], I.C[2])); break;
    case 4: o = sv(v3(I.B[1], I.B[4], I.B[7]), v3(I.C[1], I.C[3], I.C[4])); break;
    default: o = sv(v3(I.B[2], I.B[5], I.B[8]), v3(I.C[2], I.C[4], I.C[5])); break;
  }
  return o;
}
__device__ __forceinline__ void sym_add(Sym6 &I, const Sym6 &J) {
#pragma unroll
  for (int i = 0; i < 6; ++i) { I.A[i] += J.A[i]; I.C[i] += J.C[i]; }
#pragma unroll
  for (int i = 0; i < 9; ++i) I.B[i] += J.B[i];
}
// I - U U^T / D
__device__ __forceinline__ void sym_rank1(Sym6 &I, SV U, float dinv) {
  const float u[6] = {U.a.x, U.a.y, U.a.z, U.b.x, U.b.y, U.b.z};
  const int sx[6] = {0, 0, 0, 1, 1, 2}, sy[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    I.A[i] -= u[sx[i]] * u[sy[i]] * dinv;
    I.C[i] -= u[3 + sx[i]] * u[3 + sy[i]] * dinv;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) I.B[3 * r + c] -= u[r] * u[3 + c] * dinv;
}
// The translation part of X^T I X for a child -> parent transform X = (R, r)
// once the blocks are turned (A' = R A R^T, B' = R B R^T, C' = R C R^T):
// A'' = A' + rx B'^T - B' rx - rx C' rx,  B'' = B' + rx C',  C'' = C'.
__device__ __forceinline__ Sym6 shift_inertia(const Sym6 &R, V3f r) {
  // rx C' (3x3): row i = r x (column of C')... compute M = rx C' explicitly
  const float *C = R.C;
  const float Cf[9] = {C[0], C[1], C[2], C[1], C[3], C[4], C[2], C[4], C[5]};
  float M[9];  // M = rx C'
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const V3f col = v3(Cf[c], Cf[3 + c], Cf[6 + c]);
    const V3f m = cross(r, col);
    M[c] = m.x; M[3 + c] = m.y; M[6 + c] = m.z;
  }
  // N = rx B'^T ; P = B' rx ; Q = M rx = rx C' rx
  float N[9], P[9], Q[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const V3f bt = v3(R.B[3 * c], R.B[3 * c + 1], R.B[3 * c + 2]);  // column c of B'^T = row c of B'
    const V3f n = cross(r, bt);
    N[c] = n.x; N[3 + c] = n.y; N[6 + c] = n.z;
  }
  // P = B' rx: row i of P = (row i of B') rx = -(r x row_i)^T ... use P_ij = sum_k B_ik rx_kj
  const float rx[9] = {0.0f, -r.z, r.y, r.z, 0.0f, -r.x, -r.y, r.x, 0.0f};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      P[3 * i + j] = R.B[3 * i] * rx[j] + R.B[3 * i + 1] * rx[3 + j] + R.B[3 * i + 2] * rx[6 + j];
      Q[3 * i + j] = M[3 * i] * rx[j] + M[3 * i + 1] * rx[3 + j] + M[3 * i + 2] * rx[6 + j];
    }
  Sym6 O;
  const int sx[6] = {0, 0, 0, 1, 1, 2}, sy[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int a = 3 * sx[i] + sy[i];
    O.A[i] = R.A[i] + N[a] - P[a] - Q[a];
    O.C[i] = R.C[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) O.B[i] = R.B[i] + M[i];
  return O;
}

// Spatial inertia of body j about its origin: A = Ic + m (|c|^2 1 - c c^T), B = m cx, C = m 1.
__device__ __forceinline__ Sym6 body_inertia(CScene &sc, int j) {
  const float m = sc.b_mass[j];
  const float hx = sc.b_half[j][0], hy = sc.b_half[j][1], hz = sc.b_half[j][2];
  const V3f c = v3(sc.b_com[j][0], sc.b_com[j][1], sc.b_com[j][2]);
  const float cc = dot(c, c);
  Sym6 I;
  I.A[0] = m * (hy * hy + hz * hz) / 3.0f + m * (cc - c.x * c.x);
  I.A[1] = -m * c.x * c.y;
  I.A[2] = -m * c.x * c.z;
  I.A[3] = m * (hx * hx + hz * hz) / 3.0f + m * (cc - c.y * c.y);
  I.A[4] = -m * c.y * c.z;
  I.A[5] = m * (hx * hx + hy * hy) / 3.0f + m * (cc - c.z * c.z);
  I.B[0] = 0.0f; I.B[1] = -m * c.z; I.B[2] = m * c.y;
  I.B[3] = m * c.z; I.B[4] = 0.0f; I.B[5] = -m * c.x;
  I.B[6] = -m * c.y; I.B[7] = m * c.x; I.B[8] = 0.0f;
  I.C[0] = m; I.C[1] = 0.0f; I.C[2] = 0.0f; I.C[3] = m; I.C[4] = 0.0f; I.C[5] = m;
  return I;
}

__device__ __forceinline__ int parent_of(int j) { return j <= PALM ? j - 1 : PALM; }
// motion subspace: index of the nonzero entry (0..5) and its sign
__device__ __forceinline__ int s_index(CScene &sc, int j) { return (sc.j_type[j] == 0 ? 0 : 3) + sc.j_axis[j] % 3; }
__device__ __forceinline__ float s_sign(CScene &sc, int j) { return sc.j_axis[j] < 3 ? 1.0f : -1.0f; }
__device__ __forceinline__ SV s_vec(CScene &sc, int j, float x) {
  const int k = s_index(sc, j);
  const float v = s_sign(sc, j) * x;
  return sv(v3(k == 0 ? v : 0.0f, k == 1 ? v : 0.0f, k == 2 ? v : 0.0f),
            v3(k == 3 ? v : 0.0f, k == 4 ? v : 0.0f, k == 5 ? v : 0.0f));
}
__device__ __forceinline__ float s_comp(CScene &sc, int j, SV x) {
  const int k = s_index(sc, j);
  const float c = k == 0 ? x.a.x : k == 1 ? x.a.y : k == 2 ? x.a.z : k == 3 ? x.b.x : k == 4 ? x.b.y : x.b.z;
  return s_sign(sc, j) * c;
}

// ---- joints about / along a principal axis ----
// Joint j at q rotates about (revolute) or slides along (prismatic) the
// principal axis e_k, k = j_axis % 3, with sign sg = +-1.  Its rotation R
// (child -> parent) turns by sg q about e_k: with (I, J) = (k+1, k+2) mod 3,
// R e_I = c e_I + s e_J, R e_J = -s e_I + c e_J, R e_k = e_k, where c = cos q
// and s = sg sin q (c = 1, s = 0 for a prismatic joint).  r is the child
// origin in parent coordinates.  Every product with R then touches two
// components only; the axis is the same for the whole wave, so the
// specialised code is chosen by a uniform branch.
struct JT {
  int k;
  float c, s;
  V3f r;
};
__device__ __forceinline__ JT joint_of(CScene &sc, int j, float q) {
  JT J;
  const int ax = sc.j_axis[j];
  J.k = ax % 3;
  const float sg = ax < 3 ? 1.0f : -1.0f;
  V3f r = v3(sc.j_origin[j][0], sc.j_origin[j][1], sc.j_origin[j][2]);
  if (sc.j_type[j] == 0) {
    float sn, cs;
    sincos_rad(q, &sn, &cs);
    J.c = cs;
    J.s = sg * sn;
  } else {
    J.c = 1.0f;
    J.s = 0.0f;
    const float d = sg * q;
    if (J.k == 0) r.x += d;
    else if (J.k == 1) r.y += d;
    else r.z += d;
  }
  J.r = r;
  return J;
}
template <int M> __device__ __forceinline__ float cget(const V3f &v) { return M == 0 ? v.x : (M == 1 ? v.y : v.z); }
template <int M> __device__ __forceinline__ void cset(V3f &v, float x) {
  if (M == 0) v.x = x;
  else if (M == 1) v.y = x;
  else v.z = x;
}
// R v for the rotation about e_K by (c, s)
template <int K> __device__ __forceinline__ V3f rot_k(float c, float s, V3f v) {
  constexpr int I = (K + 1) % 3, J = (K + 2) % 3;
  V3f o;
  cset<I>(o, c * cget<I>(v) - s * cget<J>(v));
  cset<J>(o, s * cget<I>(v) + c * cget<J>(v));
  cset<K>(o, cget<K>(v));
  return o;
}
// index of (m, n) in the packed symmetric 3x3 (xx xy xz yy yz zz)
__host__ __device__ constexpr int sidx(int m, int n) {
  return m <= n ? (m == 0 ? n : (m == 1 ? 2 + n : 5)) : (n == 0 ? m : (n == 1 ? 2 + m : 5));
}
// child -> parent motion transform: X m = [E w; E (v - r x w)] with E = R^T
template <int K> __device__ __forceinline__ SV x_motion_k(const JT &J, SV m) {
  return sv(rot_k<K>(J.c, -J.s, m.a), rot_k<K>(J.c, -J.s, m.b - cross(J.r, m.a)));
}
// X^T f = [R n + r x R f; R f]
template <int K> __device__ __forceinline__ SV x_force_T_k(const JT &J, SV f) {
  const V3f ff = rot_k<K>(J.c, J.s, f.b);
  return sv(rot_k<K>(J.c, J.s, f.a) + cross(J.r, ff), ff);
}
// Rp R (a world rotation times the joint rotation): columns I and J mix
template <int K> __device__ __forceinline__ V3f row_rot_k(V3f p, float c, float s) {
  constexpr int I = (K + 1) % 3, J = (K + 2) % 3;
  V3f o;
  cset<I>(o, c * cget<I>(p) + s * cget<J>(p));
  cset<J>(o, c * cget<J>(p) - s * cget<I>(p));
  cset<K>(o, cget<K>(p));
  return o;
}
template <int K> __device__ __forceinline__ M3f rot_right_k(const M3f &P, float c, float s) {
  M3f O;
  O.r0 = row_rot_k<K>(P.r0, c, s);
  O.r1 = row_rot_k<K>(P.r1, c, s);
  O.r2 = row_rot_k<K>(P.r2, c, s);
  return O;
}
// X^T I X: the blocks turned by R (R S R^T: only the I, J rows and columns
// mix), then the shift by r
// R S R^T for a packed symmetric block S (only the I, J rows and columns mix)
template <int K>
__device__ __forceinline__ void rot_sym_k(float c, float s, float cc, float ss, float cs, const float (&X)[6],
                                          float (&O)[6]) {
  constexpr int I = (K + 1) % 3, J = (K + 2) % 3;
  constexpr int II = sidx(I, I), JJ = sidx(J, J), IJ = sidx(I, J), IK = sidx(I, K), JK = sidx(J, K), KK = sidx(K, K);
  const float sii = X[II], sjj = X[JJ], sij = X[IJ], sik = X[IK], sjk = X[JK];
  O[II] = cc * sii - 2.0f * cs * sij + ss * sjj;
  O[JJ] = ss * sii + 2.0f * cs * sij + cc * sjj;
  O[IJ] = cs * (sii - sjj) + (cc - ss) * sij;
  O[IK] = c * sik - s * sjk;
  O[JK] = s * sik + c * sjk;
  O[KK] = X[KK];
}
template <int K> __device__ __forceinline__ Sym6 congruence_k(const JT &Jt, const Sym6 &S) {
  constexpr int I = (K + 1) % 3, J = (K + 2) % 3;
  const float c = Jt.c, s = Jt.s, cc = c * c, ss = s * s, cs = c * s;
  Sym6 R;
  rot_sym_k<K>(c, s, cc, ss, cs, S.A, R.A);
  rot_sym_k<K>(c, s, cc, ss, cs, S.C, R.C);
  // general block: P = R B (rows I, J mix), then P R^T (columns I, J mix)
  float P[9];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    P[3 * I + n] = c * S.B[3 * I + n] - s * S.B[3 * J + n];
    P[3 * J + n] = s * S.B[3 * I + n] + c * S.B[3 * J + n];
    P[3 * K + n] = S.B[3 * K + n];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    R.B[3 * m + I] = c * P[3 * m + I] - s * P[3 * m + J];
    R.B[3 * m + J] = s * P[3 * m + I] + c * P[3 * m + J];
    R.B[3 * m + K] = P[3 * m + K];
  }
  return shift_inertia(R, Jt.r);
}
#define CEM_AXIS_CASES(k, CALL)          \
  switch (k) {                           \
    case 0: { constexpr int K = 0; CALL; } \
    case 1: { constexpr int K = 1; CALL; } \
    default: { constexpr int K = 2; CALL; } \
  }
__device__ __forceinline__ SV x_motion(const JT &J, SV m) { CEM_AXIS_CASES(J.k, return x_motion_k<K>(J, m)) }
__device__ __forceinline__ SV x_force_T(const JT &J, SV f) { CEM_AXIS_CASES(J.k, return x_force_T_k<K>(J, f)) }
__device__ __forceinline__ M3f rot_right(const M3f &P, const JT &J) { CEM_AXIS_CASES(J.k, return rot_right_k<K>(P, J.c, J.s)) }
template <int K> struct AxisK {
  static constexpr int value = K;
};
template <bool B> struct BoolK {
  static constexpr bool value = B;
};
__device__ __forceinline__ V3f col(const M3f &R, int k);

// World poses of bodies 0..PALM (chain) for the arm kinematics.
__device__ __forceinline__ void chain_fk(CScene &sc, const float *q, M3f *Rw, V3f *pw) {
  M3f Rp;
  Rp.r0 = v3(1.0f, 0.0f, 0.0f); Rp.r1 = v3(0.0f, 1.0f, 0.0f); Rp.r2 = v3(0.0f, 0.0f, 1.0f);
  V3f pp = v3(0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int j = 0; j <= PALM; ++j) {
    const JT J = joint_of(sc, j, q[j]);
    pp = pp + mul(Rp, J.r);
    Rp = rot_right(Rp, J);
    Rw[j] = Rp;
    pw[j] = pp;
  }
}

__device__ __forceinline__ V3f ee_point(CScene &sc, const M3f &Rp, V3f pp) {
  return pp + mul(Rp, v3(sc.ee_offset[0], sc.ee_offset[1], sc.ee_offset[2]));
}

__device__ __forceinline__ float smooth01(float x) {
  const float c = fminf(1.0f, fmaxf(0.0f, x));
  return c * c * (3.0f - 2.0f * c);
}
__device__ __forceinline__ float wrap_pi(float a) {
  const float k = floorf((a + 3.14159265358979f) * 0.159154943091895f);
  return a - k * 6.28318530717959f;
}

// Static box k pose: Rz(yaw) Ry(pitch).
__device__ __forceinline__ M3f static_rot(CScene &sc, int k) {
  float sy, cy, sp, cp;
  sincosf(sc.st_yaw[k], &sy, &cy);
  sincosf(sc.st_pitch[k], &sp, &cp);
  M3f R;
  R.r0 = v3(cy * cp, -sy, cy * sp);
  R.r1 = v3(sy * cp, cy, sy * sp);
  R.r2 = v3(-sp, 0.0f, cp);
  return R;
}

// ---- box-box contact (vertex-face both ways) ----
// A box: centre p, rotation R (box -> world), half extents h.
struct Box {
  V3f p;
  M3f R;
  V3f h;
};
__device__ __forceinline__ V3f col(const M3f &R, int k) {
  return k == 0 ? v3(R.r0.x, R.r1.x, R.r2.x) : (k == 1 ? v3(R.r0.y, R.r1.y, R.r2.y) : v3(R.r0.z, R.r1.z, R.r2.z));
}
__device__ __forceinline__ V3f vabs(V3f a) { return v3(fabsf(a.x), fabsf(a.y), fabsf(a.z)); }
// Box A seen from box B: M = RB^T RA (A's axes in B's frame), t = RB^T (pA - pB).
struct Rel {
  M3f M;
  V3f t;
};
__device__ __forceinline__ Rel rel_of(const Box &A, const Box &B) {
  const V3f b0 = col(B.R, 0), b1 = col(B.R, 1), b2 = col(B.R, 2);
  const V3f a0 = col(A.R, 0), a1 = col(A.R, 1), a2 = col(A.R, 2);
  Rel r;
  r.M.r0 = v3(dot(b0, a0), dot(b0, a1), dot(b0, a2));
  r.M.r1 = v3(dot(b1, a0), dot(b1, a1), dot(b1, a2));
  r.M.r2 = v3(dot(b2, a0), dot(b2, a1), dot(b2, a2));
  r.t = mulT(B.R, A.p - B.p);
  return r;
}
// rel_of for a box B whose rotation is the identity: M = RA, t = pA - pB (the
// same values, the products by exact ones and zeros left out).
__device__ __forceinline__ Rel rel_of_axis(const Box &A, const Box &B) {
  Rel r;
  r.M = A.R;
  r.t = A.p - B.p;
  return r;
}
// B seen from A: M^T and -M^T t.
__device__ __forceinline__ Rel rel_swap(const Rel &r) {
  Rel o;
  o.M.r0 = col(r.M, 0);
  o.M.r1 = col(r.M, 1);
  o.M.r2 = col(r.M, 2);
  o.t = -mulT(r.M, r.t);
  return o;
}
// True when one of the six face normals separates the boxes: then no vertex
// of either lies inside the other, so the vertex-face tests would find nothing.
__device__ __forceinline__ bool face_separated(const Rel &r, V3f hA, V3f hB) {
  const V3f m0 = vabs(r.M.r0), m1 = vabs(r.M.r1), m2 = vabs(r.M.r2);
  const V3f ta = vabs(mulT(r.M, r.t));
  return fabsf(r.t.x) > hB.x + dot(m0, hA) || fabsf(r.t.y) > hB.y + dot(m1, hA) || fabsf(r.t.z) > hB.z + dot(m2, hA) ||
         ta.x > hA.x + (m0.x * hB.x + m1.x * hB.y + m2.x * hB.z) ||
         ta.y > hA.y + (m0.y * hB.x + m1.y * hB.y + m2.y * hB.z) ||
         ta.z > hA.z + (m0.z * hB.x + m1.z * hB.y + m2.z * hB.z);
}
// False when no corner of box B can lie inside box A (r = rel_of(A, B)):
// B's corners sit at +-hB_i on each of B's axes, and A lies within
// |x_i - t_i| <= sum_j |M_ij| hA_j there, so a corner is out of reach when
// that interval stops short of hB_i.  The 0.1 mm margin is far above the
// FP32 rounding of these positions, so the corner tests this rejects would
// have found no corner inside: skipping them changes no contact.
__device__ __forceinline__ bool corners_reach(const Rel &r, V3f hA, V3f hB) {
  constexpr float MARGIN = 1e-4f;
  const V3f m0 = vabs(r.M.r0), m1 = vabs(r.M.r1), m2 = vabs(r.M.r2);
  return !(fabsf(r.t.x) + dot(m0, hA) + MARGIN < hB.x || fabsf(r.t.y) + dot(m1, hA) + MARGIN < hB.y ||
           fabsf(r.t.z) + dot(m2, hA) + MARGIN < hB.z);
}
// Vertex-face: the vertices of box A strictly inside box B (r = rel_of(A, B),
// hb B's half extents), each handed over in B's frame: f(xb, ax, sgn, d) with
// xb the vertex relative to B's centre, sgn e_ax the outward normal of B's
// nearest face and d the distance to it, in ascending vertex order (faces +x
// -x +y -y +z -z, first on ties).  The caller forms the force in B's frame
// and rotates its sums once per pair.  Vertices are built in B's frame from
// the scaled axes of A.  The inside test runs for all eight; the face search
// and the contact then run once per inside vertex of a lane, so lanes whose
// inside vertices differ share passes (the wave runs as many passes as its
// lane with the most vertices inside, not one per vertex index).  Only the
// vertices in `vmask` (bit i: vertex i) are taken.
template <class F>
__device__ __forceinline__ void verts_in_box_b(const Rel &r, V3f hA, V3f hb, F &&f, unsigned vmask = 0xFFu) {
  const V3f c0 = hA.x * col(r.M, 0), c1 = hA.y * col(r.M, 1), c2 = hA.z * col(r.M, 2);
  unsigned inside = 0u;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const V3f xb = (r.t + ((i & 4) ? c2 : -c2) + ((i & 2) ? c1 : -c1)) + ((i & 1) ? c0 : -c0);
    if (fabsf(xb.x) < hb.x && fabsf(xb.y) < hb.y && fabsf(xb.z) < hb.z) inside |= 1u << i;
  }
  inside &= vmask;
  while (inside != 0u) {  // at most eight passes
    const int i = __builtin_ctz(inside);
    inside &= inside - 1u;
    // the vertex again, as ((t +- c2) +- c1) +- c0: a product with +-1 is
    // exact, so each fused step rounds as the sum above does
    const float s0 = (i & 1) ? 1.0f : -1.0f, s1 = (i & 2) ? 1.0f : -1.0f, s2 = (i & 4) ? 1.0f : -1.0f;
    const V3f xb = v3(fmaf(s0, c0.x, fmaf(s1, c1.x, fmaf(s2, c2.x, r.t.x))),
                      fmaf(s0, c0.y, fmaf(s1, c1.y, fmaf(s2, c2.y, r.t.y))),
                      fmaf(s0, c0.z, fmaf(s1, c1.z, fmaf(s2, c2.z, r.t.z))));
    // nearest face: per axis the lesser of h - x and h + x is h - |x| (the
    // same rounded value); the first axis of least depth, and on it the -
    // face only where h + x < h - x, so ties go to the + face
    const float dx = hb.x - fabsf(xb.x), dy = hb.y - fabsf(xb.y), dz = hb.z - fabsf(xb.z);
    const bool ly = dy < dx;
    int ax = ly ? 1 : 0;
    float dmin = ly ? dy : dx;
    const bool lz = dz < dmin;
    ax = lz ? 2 : ax;
    dmin = lz ? dz : dmin;
    const float xa = ax == 0 ? xb.x : (ax == 1 ? xb.y : xb.z);
    const float ha = ax == 0 ? hb.x : (ax == 1 ? hb.y : hb.z);
    f(xb, ax, ha + xa < ha - xa ? -1.0f : 1.0f, dmin);
  }
}

__device__ __forceinline__ Box static_box(CScene &sc, CConsts &k, int b) {
  Box B;
  B.p = v3(sc.st_center[b][0], sc.st_center[b][1], sc.st_center[b][2]);
  B.h = v3(sc.st_half[b][0], sc.st_half[b][1], sc.st_half[b][2]);
  const __attribute__((address_space(4))) float *m = k.st_R[b];
  B.R.r0 = v3(m[0], m[1], m[2]);
  B.R.r1 = v3(m[3], m[4], m[5]);
  B.R.r2 = v3(m[6], m[7], m[8]);
  return B;
}
__device__ __forceinline__ Sym6 inertia_of(CConsts &k, int j) {
  Sym6 I;
  const __attribute__((address_space(4))) float *m = k.I_body[j];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    I.A[i] = m[i];
    I.C[i] = m[15 + i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) I.B[i] = m[6 + i];
  return I;
}

enum : int { MOVE = 0, PICK = 1, PLACE = 2, PUSH = 3 };
// The plan's parameter row as four named 4-vectors (one per action), so that
// choosing the active action's parameters is a value select, not an indexed load.
struct Params4 {
  float v[4][4];
};
__device__ __forceinline__ void action_params(const Params4 &zp, int a, float (&pz)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float p0 = zp.v[0][i], p1 = zp.v[1][i], p2 = zp.v[2][i], p3 = zp.v[3][i];
    pz[i] = a == 0 ? p0 : (a == 1 ? p1 : (a == 2 ? p2 : p3));
  }
}
// Action a of the plan: pick-and-place = move, pick, move, place;
// move-push = move, push (the push takes parameter blocks 1 and 2).
__device__ __forceinline__ int act_kind(bool pnp, int a) {
  return (a == 0 || a == 2) ? MOVE : (a == 1 ? (pnp ? PICK : PUSH) : PLACE);
}

}  // namespace
}  // namespace cem
