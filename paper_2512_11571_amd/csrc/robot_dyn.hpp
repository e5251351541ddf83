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

// Parent -> child transform: E (rotation parent->child coords) and r (child
// origin in parent coords).  X m = [E w; E (v - r x w)];  X^T f = [E^T n + r x E^T f; E^T f].
struct Xf {
  M3f E;
  V3f r;
};
__device__ __forceinline__ SV x_motion(const Xf &X, SV m) { return sv(mul(X.E, m.a), mul(X.E, m.b - cross(X.r, m.a))); }
__device__ __forceinline__ SV x_force_T(const Xf &X, SV f) {
  const V3f n = mulT(X.E, f.a), ff = mulT(X.E, f.b);
  return sv(n + cross(X.r, ff), ff);
}

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
// k >= 3 -> [B e_j; C e_j] (B e_j = column j of B), j = k - 3
__device__ __forceinline__ SV sym_col(const Sym6 &I, int k) {
  if (k < 3) {
    const int c0 = k == 0 ? 0 : (k == 1 ? 1 : 2), c1 = k == 0 ? 1 : (k == 1 ? 3 : 4), c2 = k == 0 ? 2 : (k == 1 ? 4 : 5);
    return sv(v3(I.A[c0], I.A[c1], I.A[c2]), v3(I.B[3 * k], I.B[3 * k + 1], I.B[3 * k + 2]));
  }
  const int j = k - 3;
  const int c0 = j == 0 ? 0 : (j == 1 ? 1 : 2), c1 = j == 0 ? 1 : (j == 1 ? 3 : 4), c2 = j == 0 ? 2 : (j == 1 ? 4 : 5);
  return sv(v3(I.B[j], I.B[3 + j], I.B[6 + j]), v3(I.C[c0], I.C[c1], I.C[c2]));
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
// S' = E^T S E for symmetric S (3x3) -- rotation of a block into the parent frame
__device__ __forceinline__ void rot_sym(const M3f &E, const float *S, float *O) {
  // columns of E are E e_k; O = E^T S E, O_ij = (E e_i)^T S (E e_j)
  const V3f e0 = v3(E.r0.x, E.r1.x, E.r2.x), e1 = v3(E.r0.y, E.r1.y, E.r2.y), e2 = v3(E.r0.z, E.r1.z, E.r2.z);
  const V3f s0 = symv(S, e0), s1 = symv(S, e1), s2 = symv(S, e2);
  O[0] = dot(e0, s0); O[1] = dot(e0, s1); O[2] = dot(e0, s2);
  O[3] = dot(e1, s1); O[4] = dot(e1, s2); O[5] = dot(e2, s2);
}
__device__ __forceinline__ void rot_gen(const M3f &E, const float *B, float *O) {
  const V3f e0 = v3(E.r0.x, E.r1.x, E.r2.x), e1 = v3(E.r0.y, E.r1.y, E.r2.y), e2 = v3(E.r0.z, E.r1.z, E.r2.z);
  const V3f b0 = matv(B, e0), b1 = matv(B, e1), b2 = matv(B, e2);
  O[0] = dot(e0, b0); O[1] = dot(e0, b1); O[2] = dot(e0, b2);
  O[3] = dot(e1, b0); O[4] = dot(e1, b1); O[5] = dot(e1, b2);
  O[6] = dot(e2, b0); O[7] = dot(e2, b1); O[8] = dot(e2, b2);
}
// X^T I X: rotate the blocks (A' = E^T A E, B' = E^T B E, C' = E^T C E), then shift by r:
// A'' = A' + rx B'^T - B' rx - rx C' rx,  B'' = B' + rx C',  C'' = C'
__device__ __forceinline__ Sym6 congruence(const Xf &X, const Sym6 &I) {
  Sym6 R;
  rot_sym(X.E, I.A, R.A);
  rot_gen(X.E, I.B, R.B);
  rot_sym(X.E, I.C, R.C);
  const V3f r = X.r;
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

__device__ __forceinline__ V3f unit_axis(int a) {
  const float s = a < 3 ? 1.0f : -1.0f;
  const int k = a % 3;
  return v3(k == 0 ? s : 0.0f, k == 1 ? s : 0.0f, k == 2 ? s : 0.0f);
}

// Joint j at coordinate q (with s = sin q, c = cos q for a revolute joint):
// rotation R (child -> parent) and child origin r (parent coords).
__device__ __forceinline__ void joint_tf_sc(CScene &sc, int j, float q, float s, float c, M3f &R, V3f &r) {
  const V3f o = v3(sc.j_origin[j][0], sc.j_origin[j][1], sc.j_origin[j][2]);
  const V3f a = unit_axis(sc.j_axis[j]);
  if (sc.j_type[j] == 0) {
    const float t = 1.0f - c;
    R.r0 = v3(c + a.x * a.x * t, a.x * a.y * t - a.z * s, a.x * a.z * t + a.y * s);
    R.r1 = v3(a.y * a.x * t + a.z * s, c + a.y * a.y * t, a.y * a.z * t - a.x * s);
    R.r2 = v3(a.z * a.x * t - a.y * s, a.z * a.y * t + a.x * s, c + a.z * a.z * t);
    r = o;
  } else {
    R.r0 = v3(1.0f, 0.0f, 0.0f);
    R.r1 = v3(0.0f, 1.0f, 0.0f);
    R.r2 = v3(0.0f, 0.0f, 1.0f);
    r = o + q * a;
  }
}
__device__ __forceinline__ void joint_tf(CScene &sc, int j, float q, M3f &R, V3f &r) {
  float s = 0.0f, c = 1.0f;
  if (sc.j_type[j] == 0) sincos_rad(q, &s, &c);
  joint_tf_sc(sc, j, q, s, c, R, r);
}
__device__ __forceinline__ M3f transpose3(const M3f &R) {
  M3f T;
  T.r0 = v3(R.r0.x, R.r1.x, R.r2.x);
  T.r1 = v3(R.r0.y, R.r1.y, R.r2.y);
  T.r2 = v3(R.r0.z, R.r1.z, R.r2.z);
  return T;
}
__device__ __forceinline__ M3f matmul3(const M3f &A, const M3f &B) {
  const M3f Bt = transpose3(B);
  M3f C;
  C.r0 = v3(dot(A.r0, Bt.r0), dot(A.r0, Bt.r1), dot(A.r0, Bt.r2));
  C.r1 = v3(dot(A.r1, Bt.r0), dot(A.r1, Bt.r1), dot(A.r1, Bt.r2));
  C.r2 = v3(dot(A.r2, Bt.r0), dot(A.r2, Bt.r1), dot(A.r2, Bt.r2));
  return C;
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

// World poses of bodies 0..PALM (chain) for the arm kinematics.
__device__ __forceinline__ void chain_fk(CScene &sc, const float *q, M3f *Rw, V3f *pw) {
  M3f Rp;
  Rp.r0 = v3(1.0f, 0.0f, 0.0f); Rp.r1 = v3(0.0f, 1.0f, 0.0f); Rp.r2 = v3(0.0f, 0.0f, 1.0f);
  V3f pp = v3(0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int j = 0; j <= PALM; ++j) {
    M3f R;
    V3f r;
    joint_tf(sc, j, q[j], R, r);
    pp = pp + mul(Rp, r);
    Rp = matmul3(Rp, R);
    Rw[j] = Rp;
    pw[j] = pp;
  }
}

__device__ __forceinline__ V3f ee_point(CScene &sc, const M3f &Rp, V3f pp) {
  return pp + mul(Rp, v3(sc.ee_offset[0], sc.ee_offset[1], sc.ee_offset[2]));
}

// Damped least squares on the arm joints 3..8 toward (pt, Rt):
// dq = J^T (J J^T + lambda^2 I)^-1 e, e = (pt - p_ee, 1/2 sum_k r_k x rt_k).
__device__ __forceinline__ void ik_dls(CScene &sc, float *q, V3f pt, const M3f &Rt) {
  const float lam2 = sc.ik_lambda * sc.ik_lambda;
  for (int it = 0; it < sc.ik_iters; ++it) {
    M3f Rw[PALM + 1];
    V3f pw[PALM + 1];
    chain_fk(sc, q, Rw, pw);
    const V3f pe = ee_point(sc, Rw[PALM], pw[PALM]);
    const V3f ep = pt - pe;
    const M3f &Re = Rw[PALM];
    const V3f eo = cross(v3(Re.r0.x, Re.r1.x, Re.r2.x), v3(Rt.r0.x, Rt.r1.x, Rt.r2.x)) +
                   cross(v3(Re.r0.y, Re.r1.y, Re.r2.y), v3(Rt.r0.y, Rt.r1.y, Rt.r2.y)) +
                   cross(v3(Re.r0.z, Re.r1.z, Re.r2.z), v3(Rt.r0.z, Rt.r1.z, Rt.r2.z));
    const float e[6] = {ep.x, ep.y, ep.z, 0.5f * eo.x, 0.5f * eo.y, 0.5f * eo.z};
    float J[6][NARM];
#pragma unroll
    for (int c = 0; c < NARM; ++c) {
      const int j = ARM0 + c;
      const V3f z = mul(Rw[j], unit_axis(sc.j_axis[j]));
      const V3f jv = cross(z, pe - pw[j]);
      J[0][c] = jv.x; J[1][c] = jv.y; J[2][c] = jv.z;
      J[3][c] = z.x; J[4][c] = z.y; J[5][c] = z.z;
    }
    float A[6][6];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        float acc = r == c ? lam2 : 0.0f;
#pragma unroll
        for (int k = 0; k < NARM; ++k) acc += J[r][k] * J[c][k];
        A[r][c] = acc;
      }
    // Cholesky solve
    float L[6][6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float d = A[j][j];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
      const float ljj = sqrtf(d), inv = 1.0f / ljj;
      L[j][j] = ljj;
#pragma unroll
      for (int i = j + 1; i < 6; ++i) {
        float t = A[i][j];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
        L[i][j] = t * inv;
      }
    }
    float y[6], x[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      float t = e[i];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
      y[i] = t / L[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      float t = y[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) t -= L[k][i] * x[k];
      x[i] = t / L[i][i];
    }
#pragma unroll
    for (int c = 0; c < NARM; ++c) {
      float d = 0.0f;
#pragma unroll
      for (int r = 0; r < 6; ++r) d += J[r][c] * x[r];
      q[ARM0 + c] += d;
    }
  }
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
// Vertex-face: the vertices of box A strictly inside box B (r = rel_of(A, B));
// for each, depth = distance to B's nearest face, n = that face's outward
// normal (world), x = the vertex (world), calling f(x, n, d).  Faces +x -x +y
// -y +z -z, first on ties.  Vertices are built in B's frame from the scaled
// axes of A; the face search and the world-frame quantities are computed only
// where a lane has the vertex inside.
template <class F>
__device__ __forceinline__ void verts_in_box(const Rel &r, V3f hA, const Box &B, F &&f) {
  const V3f c0 = hA.x * col(r.M, 0), c1 = hA.y * col(r.M, 1), c2 = hA.z * col(r.M, 2);
  const V3f hb = B.h;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const V3f xb = (r.t + ((i & 4) ? c2 : -c2) + ((i & 2) ? c1 : -c1)) + ((i & 1) ? c0 : -c0);
    const bool in = fabsf(xb.x) < hb.x && fabsf(xb.y) < hb.y && fabsf(xb.z) < hb.z;
    if (in) {  // skipped by the whole wave when no lane has this vertex inside
      const float ds[6] = {hb.x - xb.x, hb.x + xb.x, hb.y - xb.y, hb.y + xb.y, hb.z - xb.z, hb.z + xb.z};
      int fb = 0;
      float dmin = ds[0];
#pragma unroll
      for (int k = 1; k < 6; ++k) {
        const bool lt = ds[k] < dmin;
        fb = lt ? k : fb;
        dmin = lt ? ds[k] : dmin;
      }
      const float sgn = (fb & 1) ? -1.0f : 1.0f;
      const int ax = fb >> 1;
      const V3f nl = v3(ax == 0 ? sgn : 0.0f, ax == 1 ? sgn : 0.0f, ax == 2 ? sgn : 0.0f);
      f(B.p + mul(B.R, xb), mul(B.R, nl), dmin);
    }
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
