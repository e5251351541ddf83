// Oracle: spatial-vector rigid-body dynamics of a kinematic tree.
// TEST INFRASTRUCTURE ONLY (see ref_scalar.hpp).
//
// Featherstone's notation (Rigid Body Dynamics Algorithms, 2008): motion
// vectors [w; v], force vectors [n; f], all in body coordinates; X_i is the
// transform from the parent's coordinates to body i's.  Implemented plainly
// with explicit 6x6 matrices so each step can be read off the textbook:
//   ABA  (articulated-body algorithm, forward dynamics),
//   RNEA (recursive Newton-Euler, inverse dynamics),
//   CRBA (joint-space inertia by unit-acceleration RNEA columns).
#pragma once
#include "ref_rigid.hpp"

namespace ref {

constexpr int MAXJ = 12;

// Tree description: joint j moves body j relative to body parent[j] (-1 = world).
// The joint frame sits at `origin` in the parent's body frame, with no fixed
// rotation; a revolute joint rotates about, a prismatic joint slides along,
// axis in {+x,+y,+z,-x,-y,-z} (0..5).  Body j: mass, COM (body frame) and a
// solid box of half extents `half` about the COM for its rotational inertia.
struct Tree {
  int n;
  int type[MAXJ];    // 0 revolute, 1 prismatic
  int axis[MAXJ];
  int parent[MAXJ];
  double origin[MAXJ][3];
  double mass[MAXJ], com[MAXJ][3], half[MAXJ][3];
};

template <class T> using Vec6 = T[6];
template <class T> struct Mat6 { T m[6][6]; };

template <class T> inline V3<T> axis_vec(int a) {
  const T s = a < 3 ? T(1.0) : T(-1.0);
  const int k = a % 3;
  return V3<T>(k == 0 ? s : T(0.0), k == 1 ? s : T(0.0), k == 2 ? s : T(0.0));
}

// Rotation by angle q about unit axis a (Rodrigues).
template <class T> inline M3<T> rot_axis(const V3<T> &a, T q) {
  const T c = r_cos(q), s = r_sin(q), t = T(1.0) - c;
  M3<T> R;
  R.m[0][0] = c + a.x * a.x * t;       R.m[0][1] = a.x * a.y * t - a.z * s; R.m[0][2] = a.x * a.z * t + a.y * s;
  R.m[1][0] = a.y * a.x * t + a.z * s; R.m[1][1] = c + a.y * a.y * t;       R.m[1][2] = a.y * a.z * t - a.x * s;
  R.m[2][0] = a.z * a.x * t - a.y * s; R.m[2][1] = a.z * a.y * t + a.x * s; R.m[2][2] = c + a.z * a.z * t;
  return R;
}

// Pose of body j relative to its parent: rotation Rj (child -> parent) and the
// child origin in parent coordinates.
template <class T> inline void joint_pose(const Tree &tr, int j, T q, M3<T> *Rj, V3<T> *pj) {
  const V3<T> a = axis_vec<T>(tr.axis[j]);
  const V3<T> o(T(tr.origin[j][0]), T(tr.origin[j][1]), T(tr.origin[j][2]));
  if (tr.type[j] == 0) {
    *Rj = rot_axis(a, q);
    *pj = o;
  } else {
    *Rj = eye3<T>();
    *pj = o + q * a;
  }
}

// 6x6 motion transform X = [E 0; -E rx E], E = Rj^T, r = pj (parent coords).
template <class T> inline Mat6<T> motion_X(const M3<T> &Rj, const V3<T> &r) {
  const M3<T> E = transpose(Rj);
  M3<T> rx;
  rx.m[0][0] = T(0.0); rx.m[0][1] = -r.z; rx.m[0][2] = r.y;
  rx.m[1][0] = r.z; rx.m[1][1] = T(0.0); rx.m[1][2] = -r.x;
  rx.m[2][0] = -r.y; rx.m[2][1] = r.x; rx.m[2][2] = T(0.0);
  const M3<T> Erx = matmul(E, rx);
  Mat6<T> X;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      X.m[i][j] = E.m[i][j];
      X.m[i][j + 3] = T(0.0);
      X.m[i + 3][j] = -Erx.m[i][j];
      X.m[i + 3][j + 3] = E.m[i][j];
    }
  return X;
}

template <class T> inline void mat6_vec(const Mat6<T> &A, const T *x, T *y) {
  for (int i = 0; i < 6; ++i) {
    T s = T(0.0);
    for (int j = 0; j < 6; ++j) s = s + A.m[i][j] * x[j];
    y[i] = s;
  }
}
template <class T> inline void mat6T_vec(const Mat6<T> &A, const T *x, T *y) {
  for (int i = 0; i < 6; ++i) {
    T s = T(0.0);
    for (int j = 0; j < 6; ++j) s = s + A.m[j][i] * x[j];
    y[i] = s;
  }
}
// C = A^T B A
template <class T> inline Mat6<T> congruence(const Mat6<T> &A, const Mat6<T> &B) {
  Mat6<T> BA, C;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T s = T(0.0);
      for (int k = 0; k < 6; ++k) s = s + B.m[i][k] * A.m[k][j];
      BA.m[i][j] = s;
    }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T s = T(0.0);
      for (int k = 0; k < 6; ++k) s = s + A.m[k][i] * BA.m[k][j];
      C.m[i][j] = s;
    }
  return C;
}

// Spatial cross products: v x m (motion), v x* f (force).
template <class T> inline void crm(const T *v, const T *m, T *out) {
  const V3<T> w(v[0], v[1], v[2]), vl(v[3], v[4], v[5]), a(m[0], m[1], m[2]), b(m[3], m[4], m[5]);
  const V3<T> o1 = cross(w, a), o2 = cross(w, b) + cross(vl, a);
  out[0] = o1.x; out[1] = o1.y; out[2] = o1.z; out[3] = o2.x; out[4] = o2.y; out[5] = o2.z;
}
template <class T> inline void crf(const T *v, const T *f, T *out) {
  const V3<T> w(v[0], v[1], v[2]), vl(v[3], v[4], v[5]), n(f[0], f[1], f[2]), ff(f[3], f[4], f[5]);
  const V3<T> o1 = cross(w, n) + cross(vl, ff), o2 = cross(w, ff);
  out[0] = o1.x; out[1] = o1.y; out[2] = o1.z; out[3] = o2.x; out[4] = o2.y; out[5] = o2.z;
}

// Spatial inertia about the body origin of mass m with COM c and rotational
// inertia Ic about the COM: [Ic + m cx cx^T, m cx; m cx^T, m 1].
template <class T> inline Mat6<T> body_inertia(const Tree &tr, int j) {
  const T m = T(tr.mass[j]);
  const T hx = T(tr.half[j][0]), hy = T(tr.half[j][1]), hz = T(tr.half[j][2]);
  const T Ixx = m * (hy * hy + hz * hz) / T(3.0), Iyy = m * (hx * hx + hz * hz) / T(3.0),
          Izz = m * (hx * hx + hy * hy) / T(3.0);
  const V3<T> c(T(tr.com[j][0]), T(tr.com[j][1]), T(tr.com[j][2]));
  T cx[3][3] = {{T(0.0), -c.z, c.y}, {c.z, T(0.0), -c.x}, {-c.y, c.x, T(0.0)}};
  Mat6<T> I;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      T s = T(0.0);
      for (int l = 0; l < 3; ++l) s = s + cx[i][l] * cx[k][l];  // cx cx^T
      const T ic = (i == k) ? (i == 0 ? Ixx : (i == 1 ? Iyy : Izz)) : T(0.0);
      I.m[i][k] = ic + m * s;
      I.m[i][k + 3] = m * cx[i][k];
      I.m[i + 3][k] = m * cx[k][i];
      I.m[i + 3][k + 3] = (i == k) ? m : T(0.0);
    }
  return I;
}

template <class T> inline void motion_S(const Tree &tr, int j, T *S) {
  const V3<T> a = axis_vec<T>(tr.axis[j]);
  for (int k = 0; k < 6; ++k) S[k] = T(0.0);
  const int o = tr.type[j] == 0 ? 0 : 3;
  S[o] = a.x; S[o + 1] = a.y; S[o + 2] = a.z;
}

// World poses of all bodies: R (body -> world), p (body origin).
template <class T> inline void forward_kinematics(const Tree &tr, const T *q, M3<T> *Rw, V3<T> *pw) {
  for (int j = 0; j < tr.n; ++j) {
    M3<T> Rj;
    V3<T> pj;
    joint_pose(tr, j, q[j], &Rj, &pj);
    const int p = tr.parent[j];
    if (p < 0) {
      Rw[j] = Rj;
      pw[j] = pj;
    } else {
      Rw[j] = matmul(Rw[p], Rj);
      pw[j] = pw[p] + mul(Rw[p], pj);
    }
  }
}

// Articulated-body algorithm: qdd = FD(q, qd, tau, fext) with gravity gz
// (m/s^2 along -z) entering as a fictitious base acceleration +gz z.
// fext[j] is a spatial force on body j in its own coordinates.
// vel_out (optional) receives the body spatial velocities.  Ibody (optional)
// holds the body inertias body_inertia(tr, i), which depend on the tree only,
// so a caller stepping the same tree many times builds them once.
template <class T>
inline void aba(const Tree &tr, const T *q, const T *qd, const T *tau, const T (*fext)[6], T gz, T *qdd,
                T (*vel_out)[6] = nullptr, const Mat6<T> *Ibody = nullptr) {
  const int n = tr.n;
  Mat6<T> X[MAXJ], IA[MAXJ];
  T v[MAXJ][6], c[MAXJ][6], pA[MAXJ][6], S[MAXJ][6], U[MAXJ][6], D[MAXJ], u[MAXJ], a[MAXJ][6];
  for (int i = 0; i < n; ++i) {
    M3<T> Rj;
    V3<T> pj;
    joint_pose(tr, i, q[i], &Rj, &pj);
    X[i] = motion_X(Rj, pj);
    motion_S(tr, i, S[i]);
    T vJ[6];
    for (int k = 0; k < 6; ++k) vJ[k] = S[i][k] * qd[i];
    const int p = tr.parent[i];
    if (p < 0) {
      for (int k = 0; k < 6; ++k) { v[i][k] = vJ[k]; c[i][k] = T(0.0); }
    } else {
      T xv[6];
      mat6_vec(X[i], v[p], xv);
      for (int k = 0; k < 6; ++k) v[i][k] = xv[k] + vJ[k];
      crm(v[i], vJ, c[i]);
    }
    IA[i] = Ibody ? Ibody[i] : body_inertia<T>(tr, i);
    T Iv[6], vIv[6];
    mat6_vec(IA[i], v[i], Iv);
    crf(v[i], Iv, vIv);
    for (int k = 0; k < 6; ++k) pA[i][k] = vIv[k] - (fext ? fext[i][k] : T(0.0));
  }
  for (int i = n - 1; i >= 0; --i) {
    mat6_vec(IA[i], S[i], U[i]);
    T d = T(0.0), sp = T(0.0);
    for (int k = 0; k < 6; ++k) {
      d = d + S[i][k] * U[i][k];
      sp = sp + S[i][k] * pA[i][k];
    }
    D[i] = d;
    u[i] = tau[i] - sp;
    const int p = tr.parent[i];
    if (p >= 0) {
      Mat6<T> Ia;
      for (int r = 0; r < 6; ++r)
        for (int s = 0; s < 6; ++s) Ia.m[r][s] = IA[i].m[r][s] - U[i][r] * U[i][s] / D[i];
      T Iac[6], pa[6];
      mat6_vec(Ia, c[i], Iac);
      for (int k = 0; k < 6; ++k) pa[k] = pA[i][k] + Iac[k] + U[i][k] * u[i] / D[i];
      const Mat6<T> Ip = congruence(X[i], Ia);
      for (int r = 0; r < 6; ++r)
        for (int s = 0; s < 6; ++s) IA[p].m[r][s] = IA[p].m[r][s] + Ip.m[r][s];
      T pp[6];
      mat6T_vec(X[i], pa, pp);
      for (int k = 0; k < 6; ++k) pA[p][k] = pA[p][k] + pp[k];
    }
  }
  const T a0[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), gz};
  for (int i = 0; i < n; ++i) {
    const int p = tr.parent[i];
    T ap[6];
    if (p < 0) mat6_vec(X[i], a0, ap);
    else mat6_vec(X[i], a[p], ap);
    for (int k = 0; k < 6; ++k) ap[k] = ap[k] + c[i][k];
    T Ua = T(0.0);
    for (int k = 0; k < 6; ++k) Ua = Ua + U[i][k] * ap[k];
    qdd[i] = (u[i] - Ua) / D[i];
    for (int k = 0; k < 6; ++k) a[i][k] = ap[k] + S[i][k] * qdd[i];
  }
  if (vel_out)
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < 6; ++k) vel_out[i][k] = v[i][k];
}

// Body spatial velocities v_j = X_j v_parent + S_j qd_j (body coordinates).
template <class T> inline void body_velocities(const Tree &tr, const T *q, const T *qd, T (*v)[6]) {
  for (int i = 0; i < tr.n; ++i) {
    M3<T> Rj;
    V3<T> pj;
    joint_pose(tr, i, q[i], &Rj, &pj);
    T S[6];
    motion_S(tr, i, S);
    const int p = tr.parent[i];
    T xv[6];
    if (p < 0) {
      for (int k = 0; k < 6; ++k) xv[k] = T(0.0);
    } else {
      mat6_vec(motion_X(Rj, pj), v[p], xv);
    }
    for (int k = 0; k < 6; ++k) v[i][k] = xv[k] + S[k] * qd[i];
  }
}

// Recursive Newton-Euler: tau = ID(q, qd, qdd, fext) with gravity gz.
template <class T>
inline void rnea(const Tree &tr, const T *q, const T *qd, const T *qdd, const T (*fext)[6], T gz, T *tau) {
  const int n = tr.n;
  Mat6<T> X[MAXJ];
  T v[MAXJ][6], a[MAXJ][6], f[MAXJ][6], S[MAXJ][6];
  const T a0[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), gz};
  for (int i = 0; i < n; ++i) {
    M3<T> Rj;
    V3<T> pj;
    joint_pose(tr, i, q[i], &Rj, &pj);
    X[i] = motion_X(Rj, pj);
    motion_S(tr, i, S[i]);
    T vJ[6];
    for (int k = 0; k < 6; ++k) vJ[k] = S[i][k] * qd[i];
    const int p = tr.parent[i];
    T xv[6], xa[6];
    if (p < 0) {
      for (int k = 0; k < 6; ++k) xv[k] = T(0.0);
      mat6_vec(X[i], a0, xa);
    } else {
      mat6_vec(X[i], v[p], xv);
      mat6_vec(X[i], a[p], xa);
    }
    for (int k = 0; k < 6; ++k) v[i][k] = xv[k] + vJ[k];
    T cj[6];
    crm(v[i], vJ, cj);
    for (int k = 0; k < 6; ++k) a[i][k] = xa[k] + S[i][k] * qdd[i] + cj[k];
    const Mat6<T> I = body_inertia<T>(tr, i);
    T Ia[6], Iv[6], vIv[6];
    mat6_vec(I, a[i], Ia);
    mat6_vec(I, v[i], Iv);
    crf(v[i], Iv, vIv);
    for (int k = 0; k < 6; ++k) f[i][k] = Ia[k] + vIv[k] - (fext ? fext[i][k] : T(0.0));
  }
  for (int i = n - 1; i >= 0; --i) {
    T t = T(0.0);
    for (int k = 0; k < 6; ++k) t = t + S[i][k] * f[i][k];
    tau[i] = t;
    const int p = tr.parent[i];
    if (p >= 0) {
      T fp[6];
      mat6T_vec(X[i], f[i], fp);
      for (int k = 0; k < 6; ++k) f[p][k] = f[p][k] + fp[k];
    }
  }
}

// Joint-space inertia: column j = RNEA(q, 0, e_j) without gravity or external forces.
template <class T> inline void crba(const Tree &tr, const T *q, T *M) {
  T zero[MAXJ], e[MAXJ], col[MAXJ];
  for (int i = 0; i < tr.n; ++i) zero[i] = T(0.0);
  for (int j = 0; j < tr.n; ++j) {
    for (int i = 0; i < tr.n; ++i) e[i] = i == j ? T(1.0) : T(0.0);
    rnea(tr, q, zero, e, (const T(*)[6]) nullptr, T(0.0), col);
    for (int i = 0; i < tr.n; ++i) M[i * tr.n + j] = col[i];
  }
}

}  // namespace ref
