// Evaluation step of CE optimisation (Alg. 1) for the mobile-manipulator
// pick-and-place plan (Sec. IV-A, pi_p&p without the final move to Exit):
//   move_to(x, y, psi, v) -> grasp(q) -> move_to(x, y, psi, v) -> place(x, y, z, psi)
// Problem 2 cost: dt per control step while the active action is not yet
// successful; tier 0 if every action succeeded and the object rests on the
// goal table's top at T (psi_g), 1 if every action succeeded but psi_g fails,
// 2 otherwise, 3 diverged.
//
// Each action runs from the step after the previous one ends (Problem 1,
// t_{0,i+1} = T_i + 1) until success or timeout.  Controllers: straight-line
// base reference at the commanded speed (smoothstep-timed) tracked by joint
// PD, arm joint targets from damped-least-squares IK solved on the GPU at
// action start and tracked along smoothstep joint-space blends, finger PD;
// torques clamped to inom * accel_max.
//
// Dynamics per substep: Featherstone's articulated-body algorithm in three
// passes over the fixed 11-body tree (base x, base y, base yaw, six arm
// joints, two fingers on the last arm body), with the contact forces on the
// base and finger links folded into the bias forces during the first pass;
// the object is a free box against the ground, the static boxes and the
// fingers (vertex-face both ways); semi-implicit Euler.
//
// One environment per lane, everything in registers: HBM is touched only for
// z in and (cost, tier, pose) out.  Scene constants are wave-uniform kernel
// arguments (scalar loads).
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
__device__ __forceinline__ Sym6 body_inertia(const cem_scene &sc, int j) {
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

// Joint j at coordinate q: rotation R (child -> parent) and child origin r (parent coords).
__device__ __forceinline__ void joint_tf(const cem_scene &sc, int j, float q, M3f &R, V3f &r) {
  const V3f o = v3(sc.j_origin[j][0], sc.j_origin[j][1], sc.j_origin[j][2]);
  const V3f a = unit_axis(sc.j_axis[j]);
  if (sc.j_type[j] == 0) {
    float s, c;
    sincosf(q, &s, &c);
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
__device__ __forceinline__ int s_index(const cem_scene &sc, int j) { return (sc.j_type[j] == 0 ? 0 : 3) + sc.j_axis[j] % 3; }
__device__ __forceinline__ float s_sign(const cem_scene &sc, int j) { return sc.j_axis[j] < 3 ? 1.0f : -1.0f; }
__device__ __forceinline__ SV s_vec(const cem_scene &sc, int j, float x) {
  const int k = s_index(sc, j);
  const float v = s_sign(sc, j) * x;
  return sv(v3(k == 0 ? v : 0.0f, k == 1 ? v : 0.0f, k == 2 ? v : 0.0f),
            v3(k == 3 ? v : 0.0f, k == 4 ? v : 0.0f, k == 5 ? v : 0.0f));
}
__device__ __forceinline__ float s_comp(const cem_scene &sc, int j, SV x) {
  const int k = s_index(sc, j);
  const float c = k == 0 ? x.a.x : k == 1 ? x.a.y : k == 2 ? x.a.z : k == 3 ? x.b.x : k == 4 ? x.b.y : x.b.z;
  return s_sign(sc, j) * c;
}

// World poses of bodies 0..PALM (chain) for the arm kinematics.
__device__ void chain_fk(const cem_scene &sc, const float *q, M3f *Rw, V3f *pw) {
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

__device__ __forceinline__ V3f ee_point(const cem_scene &sc, const M3f &Rp, V3f pp) {
  return pp + mul(Rp, v3(sc.ee_offset[0], sc.ee_offset[1], sc.ee_offset[2]));
}

// Damped least squares on the arm joints 3..8 toward (pt, Rt):
// dq = J^T (J J^T + lambda^2 I)^-1 e, e = (pt - p_ee, 1/2 sum_k r_k x rt_k).
__device__ void ik_dls(const cem_scene &sc, float *q, V3f pt, const M3f &Rt) {
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
__device__ __forceinline__ M3f static_rot(const cem_scene &sc, int k) {
  float sy, cy, sp, cp;
  sincosf(sc.st_yaw[k], &sy, &cy);
  sincosf(sc.st_pitch[k], &sp, &cp);
  M3f R;
  R.r0 = v3(cy * cp, -sy, cy * sp);
  R.r1 = v3(sy * cp, cy, sy * sp);
  R.r2 = v3(-sp, 0.0f, cp);
  return R;
}

// Vertex-face: vertices of box A (pa, Ra, ha) strictly inside box B (pb, Rb, hb);
// for each, depth = distance to B's nearest face, n = that face's outward
// normal (world), calling f(x, n, d).  Faces +x -x +y -y +z -z, first on ties.
template <class F>
__device__ __forceinline__ void verts_in_box(V3f pa, const M3f &Ra, V3f ha, V3f pb, const M3f &Rb, V3f hb, F &&f) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const V3f loc = v3((i & 1) ? ha.x : -ha.x, (i & 2) ? ha.y : -ha.y, (i & 4) ? ha.z : -ha.z);
    const V3f x = pa + mul(Ra, loc);
    const V3f xb = mulT(Rb, x - pb);
    const bool in = fabsf(xb.x) < hb.x && fabsf(xb.y) < hb.y && fabsf(xb.z) < hb.z;
    float ds[6] = {hb.x - xb.x, hb.x + xb.x, hb.y - xb.y, hb.y + xb.y, hb.z - xb.z, hb.z + xb.z};
    int fb = 0;
#pragma unroll
    for (int k = 1; k < 6; ++k) fb = ds[k] < ds[fb] ? k : fb;
    const float sgn = (fb & 1) ? -1.0f : 1.0f;
    const int ax = fb >> 1;
    const V3f nl = v3(ax == 0 ? sgn : 0.0f, ax == 1 ? sgn : 0.0f, ax == 2 ? sgn : 0.0f);
    f(in, x, mul(Rb, nl), ds[fb]);
  }
}

enum : int { MOVE = 0, PICK = 1, PLACE = 2 };
__device__ __forceinline__ int act_kind(int a) { return (a == 0 || a == 2) ? MOVE : (a == 1 ? PICK : PLACE); }

template <bool TRACE>
__global__ void __launch_bounds__(64) rollout_pickplace_kernel(cem_scene sc, const float *__restrict__ Z, int pop,
                                                               float *__restrict__ cost_out,
                                                               uint8_t *__restrict__ tier_out,
                                                               float *__restrict__ pose_out,
                                                               float *__restrict__ trace, int trace_steps) {
  const int env = blockIdx.x * blockDim.x + threadIdx.x;
  if (env >= pop) return;
  const float h = sc.dt / (float)sc.substeps;
  const float dt = sc.dt;
  const float g = sc.gravity;
  const float kc = sc.k_contact, damp = sc.c_contact, eps2 = sc.eps_v * sc.eps_v;
  const float wc = sc.omega_c, zeta = sc.zeta;
  const V3f ohe = v3(sc.obj_half[0], sc.obj_half[1], sc.obj_half[2]);
  const float om = sc.obj_mass, inv_om = 1.0f / om;
  const V3f oIb = v3(om * (ohe.y * ohe.y + ohe.z * ohe.z) / 3.0f, om * (ohe.x * ohe.x + ohe.z * ohe.z) / 3.0f,
                     om * (ohe.x * ohe.x + ohe.y * ohe.y) / 3.0f);
  const V3f gv = v3(0.0f, 0.0f, -g);

  float zp[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) zp[i] = Z[(long)env * 16 + i];

  float q[NJ], qd[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) { q[j] = sc.q0[j]; qd[j] = 0.0f; }
  FreeBody ob;
  ob.p = v3(sc.obj_pos0[0], sc.obj_pos0[1], sc.obj_pos0[2] - om * g / (4.0f * kc));
  {
    float s, c;
    sincosf(0.5f * sc.obj_yaw0, &s, &c);
    ob.q = Q4f{c, 0.0f, 0.0f, s};
  }
  ob.v = v3(0.0f, 0.0f, 0.0f);
  ob.w = v3(0.0f, 0.0f, 0.0f);

  // controller state
  int act = 0, t_start = 0;
  unsigned ok_bits = 0;
  float qstart[NARM + 3], qa[NARM], qb[NARM];
  V3f ptarget = v3(0.0f, 0.0f, 0.0f);
  float base_from[3], base_to[3], t_move = 1.0f;
  float Ta = sc.t_approach, Td = sc.t_descend, Tl = sc.t_lift, Tp = sc.t_transfer;
  float finger_cmd = sc.finger_open;
  bool touchL = false, touchR = false;
  int unsuccessful = 0;
  float qref[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) qref[j] = q[j];
#pragma unroll
  for (int j = 0; j < NARM; ++j) { qa[j] = 0.0f; qb[j] = 0.0f; }

  auto span = [&](const float *from, const float *to, float nominal) {
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < NARM; ++j) m = fmaxf(m, fabsf(to[j] - from[j]));
    return fmaxf(nominal, m / sc.joint_speed_max);
  };

  auto start_action = [&](int a, int t) {
    t_start = t;
#pragma unroll
    for (int j = 0; j < NARM + 3; ++j) qstart[j] = q[j];
    const float *pz = zp + 4 * a;
    const int kind = act_kind(a);
    if (kind == MOVE) {
      base_from[0] = q[0]; base_from[1] = q[1]; base_from[2] = q[2];
      const float dpsi = wrap_pi(pz[2] - q[2]);
      base_to[0] = pz[0]; base_to[1] = pz[1]; base_to[2] = q[2] + dpsi;
      const float v = fmaxf(sc.base_vmin, fminf(sc.base_vmax, pz[3]));
      const float dx = pz[0] - q[0], dy = pz[1] - q[1];
      const float L = sqrtf(dx * dx + dy * dy);
      t_move = fmaxf(fmaxf(L / v, fabsf(dpsi) / sc.base_wmax), dt);
    } else {
      M3f Rt;
      V3f pfin, pgoal;
      if (kind == PICK) {
        // grasp orientation from the normalised quaternion parameter
        float w = pz[0], x = pz[1], y = pz[2], z = pz[3];
        const float n2 = w * w + x * x + y * y + z * z;
        if (!(n2 > 1e-12f)) { w = 1.0f; x = 0.0f; y = 0.0f; z = 0.0f; }
        else {
          const float inv = 1.0f / sqrtf(n2);
          w *= inv; x *= inv; y *= inv; z *= inv;
        }
        Rt = rot_of(Q4f{w, x, y, z});
        pgoal = ob.p;
        pfin = pgoal - sc.pregrasp * v3(Rt.r0.z, Rt.r1.z, Rt.r2.z);
      } else {
        float sy, cy;
        sincosf(pz[3], &sy, &cy);
        Rt.r0 = v3(cy, sy, 0.0f);
        Rt.r1 = v3(sy, -cy, 0.0f);
        Rt.r2 = v3(0.0f, 0.0f, -1.0f);
        pfin = v3(pz[0], pz[1], pz[2]);
        pgoal = pfin;
      }
      float qq[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) qq[j] = q[j];
      ik_dls(sc, qq, pfin, Rt);
      float qaf[NARM + 3];
#pragma unroll
      for (int j = 0; j < NARM; ++j) qa[j] = qq[ARM0 + j];
      if (kind == PICK) {
        ik_dls(sc, qq, pgoal, Rt);
#pragma unroll
        for (int j = 0; j < NARM; ++j) qb[j] = qq[ARM0 + j];
        float qs[NARM];
#pragma unroll
        for (int j = 0; j < NARM; ++j) qs[j] = qstart[ARM0 + j];
        Ta = span(qs, qa, sc.t_approach);
        Td = span(qa, qb, sc.t_descend);
        Tl = span(qb, qa, sc.t_lift);
      } else {
        float qs[NARM];
#pragma unroll
        for (int j = 0; j < NARM; ++j) qs[j] = qstart[ARM0 + j];
        Tp = span(qs, qa, sc.t_transfer);
      }
      (void)qaf;
      ptarget = pfin;
    }
  };

  const int n_act = 4;
  start_action(0, 0);
  bool diverged = false;
  for (int t = 0; t < sc.horizon; ++t) {
    if (act < n_act) {
      const float tau = (float)(t - t_start) * dt;
      const int kind = act_kind(act);
      bool succ;
      if (kind == MOVE) {
        const float *pz = zp + 4 * act;
        const float dx = q[0] - pz[0], dy = q[1] - pz[1];
        succ = sqrtf(dx * dx + dy * dy) <= sc.base_tol && fabsf(wrap_pi(q[2] - pz[2])) <= sc.yaw_tol;
      } else {
        M3f Rw[PALM + 1];
        V3f pw[PALM + 1];
        chain_fk(sc, q, Rw, pw);
        const V3f pe = ee_point(sc, Rw[PALM], pw[PALM]);
        const V3f de = pe - ptarget;
        const bool near = sqrtf(dot(de, de)) <= sc.ee_tol;
        if (kind == PICK) {
          const float tend = Ta + Td + sc.t_close + Tl;
          const V3f op = mulT(Rw[PALM], ob.p - pw[PALM]);
          const bool between = op.y < q[FL] && op.y > -q[FR];
          succ = tau >= tend && touchL && touchR && between && near;
        } else {
          succ = tau >= Tp + sc.t_release && near;
        }
      }
      const float tout = kind == MOVE ? sc.timeout_move : (kind == PICK ? sc.timeout_pick : sc.timeout_place);
      if (succ || tau >= tout) {
        if (succ) ok_bits |= 1u << act;
        ++act;
        if (act < n_act) start_action(act, t);
      }
    }
    if (act < n_act) ++unsuccessful;
    if (act < n_act) {
      const float tau = (float)(t - t_start) * dt;
      const int kind = act_kind(act);
      if (kind == MOVE) {
        const float sft = smooth01(tau / t_move);
#pragma unroll
        for (int c = 0; c < 3; ++c) qref[c] = base_from[c] + sft * (base_to[c] - base_from[c]);
#pragma unroll
        for (int j = 0; j < NARM; ++j) qref[ARM0 + j] = qstart[ARM0 + j];
      } else if (kind == PICK) {
        const float Tc = sc.t_close;
#pragma unroll
        for (int c = 0; c < 3; ++c) qref[c] = qstart[c];
#pragma unroll
        for (int j = 0; j < NARM; ++j) {
          float r;
          const float s0 = qstart[ARM0 + j];
          if (tau < Ta) r = s0 + smooth01(tau / Ta) * (qa[j] - s0);
          else if (tau < Ta + Td) r = qa[j] + smooth01((tau - Ta) / Td) * (qb[j] - qa[j]);
          else if (tau < Ta + Td + Tc) r = qb[j];
          else if (tau < Ta + Td + Tc + Tl) r = qb[j] + smooth01((tau - Ta - Td - Tc) / Tl) * (qa[j] - qb[j]);
          else r = qa[j];
          qref[ARM0 + j] = r;
        }
        finger_cmd = tau < Ta + Td ? sc.finger_open : sc.finger_closed;
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) qref[c] = qstart[c];
#pragma unroll
        for (int j = 0; j < NARM; ++j) {
          const float s0 = qstart[ARM0 + j];
          qref[ARM0 + j] = tau < Tp ? s0 + smooth01(tau / Tp) * (qa[j] - s0) : qa[j];
        }
        finger_cmd = tau < Tp ? sc.finger_closed : sc.finger_open;
      }
    }
    qref[FL] = finger_cmd;
    qref[FR] = finger_cmd;

    for (int si = 0; si < sc.substeps; ++si) {
      const bool last = si == sc.substeps - 1;
      // ---- object contacts with the world (ground, static boxes) ----
      const M3f oR = rot_of(ob.q);
      Wrench W{v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f)};
      box_ground(ob, oR, ohe, kc, damp, sc.mu_ground, eps2, W);
      for (int b = 0; b < sc.n_static; ++b) {
        const M3f SR = static_rot(sc, b);
        const V3f SP = v3(sc.st_center[b][0], sc.st_center[b][1], sc.st_center[b][2]);
        const V3f SH = v3(sc.st_half[b][0], sc.st_half[b][1], sc.st_half[b][2]);
        const float mu = sc.st_ramp[b] ? sc.mu_ramp : sc.mu_static;
        verts_in_box(ob.p, oR, ohe, SP, SR, SH, [&](bool in, V3f x, V3f n, float d) {
          const V3f r = x - ob.p;
          apply(W, r, contact_force(in, n, d, ob.v + cross(ob.w, r), kc, damp, mu, eps2));
        });
        verts_in_box(SP, SR, SH, ob.p, oR, ohe, [&](bool in, V3f x, V3f n, float d) {
          const V3f r = x - ob.p;
          // A = static box, B = object: the object receives the negative
          apply(W, r, -contact_force(in, n, d, v3(0.0f, 0.0f, 0.0f) - (ob.v + cross(ob.w, r)), kc, damp, mu, eps2));
        });
      }

      // ---- ABA pass 1: kinematics, velocities, bias forces, link contacts ----
      SV c_[NJ], pA[NJ];
      M3f Rw;  // world rotation of the current chain body
      V3f pw;
      M3f Rw8;
      V3f pw8;
      SV v8;
      SV vprev = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f));
      Rw.r0 = v3(1.0f, 0.0f, 0.0f); Rw.r1 = v3(0.0f, 1.0f, 0.0f); Rw.r2 = v3(0.0f, 0.0f, 1.0f);
      pw = v3(0.0f, 0.0f, 0.0f);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int p = parent_of(j);
        M3f Rj;
        V3f rj;
        joint_tf(sc, j, q[j], Rj, rj);
        Xf X;
        X.E = transpose3(Rj);
        X.r = rj;
        const M3f Rp = (j == FL || j == FR) ? Rw8 : Rw;
        const V3f pp = (j == FL || j == FR) ? pw8 : pw;
        const SV vp = (j == FL || j == FR) ? v8 : vprev;
        const M3f Rb = matmul3(Rp, Rj);
        const V3f pb = pp + mul(Rp, rj);
        const SV vJ = s_vec(sc, j, qd[j]);
        const SV vb = (p < 0 ? sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f)) : x_motion(X, vp)) + vJ;
        c_[j] = p < 0 ? sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f)) : crm(vb, vJ);
        const Sym6 Ib = body_inertia(sc, j);
        pA[j] = crf(vb, sym_mul(Ib, vb));
        // contacts on this link (world forces -> body spatial force, subtracted from pA)
        if (j == BASEB) {
          const V3f bc = pb + mul(Rb, v3(sc.b_com[j][0], sc.b_com[j][1], sc.b_com[j][2]));
          const V3f bh = v3(sc.b_half[j][0], sc.b_half[j][1], sc.b_half[j][2]);
          SV fe = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f));
          auto link_v = [&](V3f x) {
            const V3f xb = mulT(Rb, x - pb);
            return mul(Rb, vb.b + cross(vb.a, xb));
          };
          auto link_f = [&](V3f x, V3f F) {
            const V3f Fb = mulT(Rb, F), xb = mulT(Rb, x - pb);
            fe = fe + sv(cross(xb, Fb), Fb);
          };
          for (int b = 0; b < sc.n_static; ++b) {
            const M3f SR = static_rot(sc, b);
            const V3f SP = v3(sc.st_center[b][0], sc.st_center[b][1], sc.st_center[b][2]);
            const V3f SH = v3(sc.st_half[b][0], sc.st_half[b][1], sc.st_half[b][2]);
            verts_in_box(bc, Rb, bh, SP, SR, SH, [&](bool in, V3f x, V3f n, float d) {
              link_f(x, contact_force(in, n, d, link_v(x), kc, damp, sc.mu_static, eps2));
            });
            verts_in_box(SP, SR, SH, bc, Rb, bh, [&](bool in, V3f x, V3f n, float d) {
              link_f(x, -contact_force(in, n, d, v3(0.0f, 0.0f, 0.0f) - link_v(x), kc, damp, sc.mu_static, eps2));
            });
          }
          pA[j] = pA[j] - fe;
        }
        if (j == FL || j == FR) {
          const V3f fc = pb + mul(Rb, v3(sc.b_com[j][0], sc.b_com[j][1], sc.b_com[j][2]));
          const V3f fh = v3(sc.b_half[j][0], sc.b_half[j][1], sc.b_half[j][2]);
          SV fe = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f));
          bool any = false;
          auto link_v = [&](V3f x) {
            const V3f xb = mulT(Rb, x - pb);
            return mul(Rb, vb.b + cross(vb.a, xb));
          };
          auto link_f = [&](V3f x, V3f F) {
            const V3f Fb = mulT(Rb, F), xb = mulT(Rb, x - pb);
            fe = fe + sv(cross(xb, Fb), Fb);
          };
          // finger vertices in the object (A = finger, B = object)
          verts_in_box(fc, Rb, fh, ob.p, oR, ohe, [&](bool in, V3f x, V3f n, float d) {
            const V3f ro = x - ob.p;
            const V3f F = contact_force(in, n, d, link_v(x) - (ob.v + cross(ob.w, ro)), kc, damp, sc.mu_tool, eps2);
            link_f(x, F);
            apply(W, ro, -F);
            any = any || in;
          });
          // object vertices in the finger (A = object, B = finger)
          verts_in_box(ob.p, oR, ohe, fc, Rb, fh, [&](bool in, V3f x, V3f n, float d) {
            const V3f ro = x - ob.p;
            const V3f F = contact_force(in, n, d, (ob.v + cross(ob.w, ro)) - link_v(x), kc, damp, sc.mu_tool, eps2);
            apply(W, ro, F);
            link_f(x, -F);
            any = any || in;
          });
          pA[j] = pA[j] - fe;
          if (last) {
            if (j == FL) touchL = any;
            else touchR = any;
          }
        }
        if (j <= PALM) {
          Rw = Rb;
          pw = pb;
          vprev = vb;
        }
        if (j == PALM) {
          Rw8 = Rb;
          pw8 = pb;
          v8 = vb;
        }
      }

      // ---- joint PD torques ----
      float tau_j[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const float lim = sc.j_inom[j] * sc.accel_max;
        const float u = sc.j_inom[j] * (wc * wc * (qref[j] - q[j]) - 2.0f * zeta * wc * qd[j]);
        tau_j[j] = fmaxf(-lim, fminf(lim, u));
      }

      // ---- ABA pass 2: articulated inertias, leaves to root ----
      SV U[NJ];
      float Dinv[NJ], uu[NJ];
      Sym6 IA8 = body_inertia(sc, PALM);
      SV pA8 = pA[PALM];
      Sym6 IAc;  // articulated inertia of the current chain body
      SV pAc;
#pragma unroll
      for (int j = NJ - 1; j >= 0; --j) {
        Sym6 IA;
        SV pAj;
        if (j == FL || j == FR) {
          IA = body_inertia(sc, j);
          pAj = pA[j];
        } else if (j == PALM) {
          IA = IA8;
          pAj = pA8;
        } else {
          IA = IAc;
          pAj = pAc;
        }
        const int k = s_index(sc, j);
        const SV Uj = s_sign(sc, j) * sym_col(IA, k);
        const float D = s_comp(sc, j, Uj);
        const float di = 1.0f / D;
        const float u = tau_j[j] - s_comp(sc, j, pAj);
        U[j] = Uj;
        Dinv[j] = di;
        uu[j] = u;
        if (j > 0) {
          sym_rank1(IA, Uj, di);
          const SV pa = pAj + sym_mul(IA, c_[j]) + (u * di) * Uj;
          M3f Rj;
          V3f rj;
          joint_tf(sc, j, q[j], Rj, rj);
          Xf X;
          X.E = transpose3(Rj);
          X.r = rj;
          const Sym6 Ip = congruence(X, IA);
          const SV pp = x_force_T(X, pa);
          const int p = parent_of(j);
          if (p == PALM) {
            sym_add(IA8, Ip);
            pA8 = pA8 + pp;
          } else {
            IAc = body_inertia(sc, p);
            sym_add(IAc, Ip);
            pAc = pA[p] + pp;
          }
        }
      }

      // ---- ABA pass 3: accelerations, root to leaves ----
      float qdd[NJ];
      SV a_prev = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, g));  // world: -gravity
      SV a8 = a_prev;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        M3f Rj;
        V3f rj;
        joint_tf(sc, j, q[j], Rj, rj);
        Xf X;
        X.E = transpose3(Rj);
        X.r = rj;
        const SV ap = x_motion(X, (j == FL || j == FR) ? a8 : a_prev) + c_[j];
        const float qa_ = (uu[j] - dot6(U[j], ap)) * Dinv[j];
        qdd[j] = qa_;
        const SV aj = ap + s_vec(sc, j, qa_);
        if (j <= PALM) a_prev = aj;
        if (j == PALM) a8 = aj;
      }

      // ---- integrate ----
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        qd[j] += h * qdd[j];
        q[j] += h * qd[j];
      }
      integrate(ob, W, inv_om, oIb, gv, h);
    }
    if (TRACE && t < trace_steps) {
      float *o = trace + ((long)env * trace_steps + t) * CEM_TRACE_ROBOT;
      o[0] = ob.p.x; o[1] = ob.p.y; o[2] = ob.p.z;
      o[3] = ob.q.w; o[4] = ob.q.x; o[5] = ob.q.y; o[6] = ob.q.z;
      o[7] = ob.v.x; o[8] = ob.v.y; o[9] = ob.v.z;
      o[10] = ob.w.x; o[11] = ob.w.y; o[12] = ob.w.z;
#pragma unroll
      for (int j = 0; j < NJ; ++j) { o[13 + j] = q[j]; o[24 + j] = qd[j]; }
    }
    if (!isfinite(ob.p.x) || !isfinite(q[0])) {
      diverged = true;
      break;
    }
  }
  // goal: the object rests on the goal table's top face
  bool goal = false;
  if (sc.goal_static >= 0 && sc.goal_static < sc.n_static) {
    const int b = sc.goal_static;
    const float top = sc.st_center[b][2] + sc.st_half[b][2];
    const float sp = sqrtf(dot(ob.v, ob.v));
    goal = fabsf(ob.p.x - sc.st_center[b][0]) <= sc.st_half[b][0] && fabsf(ob.p.y - sc.st_center[b][1]) <= sc.st_half[b][1] &&
           ob.p.z >= top && ob.p.z <= top + 2.0f * sc.obj_half[2] && sp < sc.rest_speed;
  }
  const float pose[7] = {ob.p.x, ob.p.y, ob.p.z, ob.q.w, ob.q.x, ob.q.y, ob.q.z};
  bool fin = !diverged;
#pragma unroll
  for (int i = 0; i < 7; ++i) fin = fin && isfinite(pose[i]);
#pragma unroll
  for (int j = 0; j < NJ; ++j) fin = fin && isfinite(q[j]) && fabsf(q[j]) < 1e3f;
  fin = fin && fabsf(ob.p.x) < 1e3f && fabsf(ob.p.y) < 1e3f && fabsf(ob.p.z) < 1e3f;
  const bool all_ok = ok_bits == 0xFu;
  const int tier = !fin ? 3 : (all_ok ? (goal ? 0 : 1) : 2);
  const float cost = fin ? sc.time_weight * dt * (float)unsuccessful : __int_as_float(0x7F800000);
  if (cost_out) cost_out[env] = cost;
  if (tier_out) tier_out[env] = (uint8_t)tier;
  if (pose_out)
#pragma unroll
    for (int i = 0; i < 7; ++i) pose_out[(long)env * 7 + i] = pose[i];
}

}  // namespace

hipError_t launch_rollout_pickplace(const cem_scene &sc, const float *Z, int pop, float *cost, uint8_t *tier,
                                    float *pose, float *trace, int trace_steps, hipStream_t s) {
  const int bs = 64;
  const dim3 grid((pop + bs - 1) / bs);
  if (trace)
    hipLaunchKernelGGL(rollout_pickplace_kernel<true>, grid, dim3(bs), 0, s, sc, Z, pop, cost, tier, pose, trace,
                       trace_steps);
  else
    hipLaunchKernelGGL(rollout_pickplace_kernel<false>, grid, dim3(bs), 0, s, sc, Z, pop, cost, tier, pose, nullptr,
                       0);
  return hipGetLastError();
}

}  // namespace cem
