// The articulated-body algorithm specialised at compile time to the robot of
// robot_model.hpp (joint axes and types, joint origins, body inertias).
//
// The generic passes read every joint's axis, type and origin and every
// body's inertia from the scene at run time and multiply through the zeros of
// the robot's structure: origins on one or two axes, centres of mass on a
// body axis, box inertias that are diagonal about the centre of mass.  Here
// those are constants: each product with a structural zero is left out (the
// helpers below expand a constant row times a vector into only its nonzero
// terms, in the generic order), the motion-subspace component and the
// principal axis of each joint are fixed, and the loops over bodies are
// unrolled.  The arithmetic that remains is the generic one's, term for term,
// without the terms that are exact zeros, so the two agree up to the rounding
// of those terms' removal (FMA groupings can differ).  The LDS rows are the
// generic layout's.
#pragma once
#include <type_traits>

#include "robot_dyn.hpp"
#include "robot_model.hpp"

namespace cem {
namespace {

// ---- compile-time loops ----
template <int B, int E, class F> __device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    sfor<B + 1, E>(f);
  }
}
// E - 1 down to B
template <int B, int E, class F> __device__ __forceinline__ void sfor_down(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, E - 1>());
    sfor_down<B, E - 1>(f);
  }
}

// ---- constant rows times vectors ----
// sum_i C::v[i] x[i] over the nonzero C::v[i], left to right (the first
// nonzero term a product, the rest fused multiply-adds); 0 when all are zero.
template <class C, int I, int N, bool S>
__device__ __forceinline__ float cdot_r(const float (&x)[N], float acc) {
  if constexpr (I == N) {
    if constexpr (S) return acc;
    else return 0.0f;
  } else {
    constexpr float c = C::v[I];
    if constexpr (c == 0.0f) return cdot_r<C, I + 1, N, S>(x, acc);
    else if constexpr (!S) return cdot_r<C, I + 1, N, true>(x, c * x[I]);
    else return cdot_r<C, I + 1, N, true>(x, fmaf(c, x[I], acc));
  }
}
template <class C, int N> __device__ __forceinline__ float cdot(const float (&x)[N]) {
  return cdot_r<C, 0, N, false>(x, 0.0f);
}
template <class C> __device__ __forceinline__ float cdot3(V3f a) {
  const float x[3] = {a.x, a.y, a.z};
  return cdot<C, 3>(x);
}

// ---- the model's constants ----
namespace rmx {
constexpr bool rev(int j) { return rm::TYPE[j] == 0; }
constexpr int kax(int j) { return rm::AXIS[j] % 3; }
constexpr float sgn(int j) { return rm::AXIS[j] < 3 ? 1.0f : -1.0f; }
constexpr int sub_idx(int j) { return (rev(j) ? 0 : 3) + kax(j); }

struct SymC {
  float A[6], B[9], C[6];
};
// body j's spatial inertia about its frame origin, as body_inertia forms it
constexpr SymC body_i(int j) {
  const float m = rm::MASS[j];
  const float hx = rm::HALF[j][0], hy = rm::HALF[j][1], hz = rm::HALF[j][2];
  const float cx = rm::COM[j][0], cy = rm::COM[j][1], cz = rm::COM[j][2];
  const float cc = cx * cx + cy * cy + cz * cz;
  SymC I{};
  I.A[0] = m * (hy * hy + hz * hz) / 3.0f + m * (cc - cx * cx);
  I.A[1] = -m * cx * cy;
  I.A[2] = -m * cx * cz;
  I.A[3] = m * (hx * hx + hz * hz) / 3.0f + m * (cc - cy * cy);
  I.A[4] = -m * cy * cz;
  I.A[5] = m * (hx * hx + hy * hy) / 3.0f + m * (cc - cz * cz);
  I.B[0] = 0.0f; I.B[1] = -m * cz; I.B[2] = m * cy;
  I.B[3] = m * cz; I.B[4] = 0.0f; I.B[5] = -m * cx;
  I.B[6] = -m * cy; I.B[7] = m * cx; I.B[8] = 0.0f;
  I.C[0] = m; I.C[1] = 0.0f; I.C[2] = 0.0f; I.C[3] = m; I.C[4] = 0.0f; I.C[5] = m;
  return I;
}
// entry (r, c) of the 6x6 [A B; B^T C] of a packed symmetric inertia
constexpr float sym_at(const SymC &I, int r, int c) {
  if (r < 3 && c < 3) return I.A[sidx(r, c)];
  if (r < 3) return I.B[3 * r + (c - 3)];
  if (c < 3) return I.B[3 * c + (r - 3)];
  return I.C[sidx(r - 3, c - 3)];
}
}  // namespace rmx

// row r of body J's inertia
template <int J, int R> struct IRow {
  static constexpr rmx::SymC I = rmx::body_i(J);
  static constexpr float v[6] = {rmx::sym_at(I, R, 0), rmx::sym_at(I, R, 1), rmx::sym_at(I, R, 2),
                                 rmx::sym_at(I, R, 3), rmx::sym_at(I, R, 4), rmx::sym_at(I, R, 5)};
};
// joint J's origin, and row / column I of its cross-product matrix [r]x
template <int J> struct Org {
  static constexpr float v[3] = {rm::ORIGIN[J][0], rm::ORIGIN[J][1], rm::ORIGIN[J][2]};
};
template <int J, int I> struct RxRow {
  static constexpr float x = rm::ORIGIN[J][0], y = rm::ORIGIN[J][1], z = rm::ORIGIN[J][2];
  static constexpr float v[3] = {I == 0 ? 0.0f : (I == 1 ? z : -y), I == 0 ? -z : (I == 1 ? 0.0f : x),
                                 I == 0 ? y : (I == 1 ? -x : 0.0f)};
};
template <int J, int I> struct RxCol {  // column I of [r]x = minus row I
  static constexpr float v[3] = {-RxRow<J, I>::v[0], -RxRow<J, I>::v[1], -RxRow<J, I>::v[2]};
};

// I_J m with I_J the body's inertia
template <int J> __device__ __forceinline__ SV body_mul(SV m) {
  const float x[6] = {m.a.x, m.a.y, m.a.z, m.b.x, m.b.y, m.b.z};
  return sv(v3(cdot<IRow<J, 0>, 6>(x), cdot<IRow<J, 1>, 6>(x), cdot<IRow<J, 2>, 6>(x)),
            v3(cdot<IRow<J, 3>, 6>(x), cdot<IRow<J, 4>, 6>(x), cdot<IRow<J, 5>, 6>(x)));
}
// the body's inertia, and the body's inertia plus S
template <int J> __device__ __forceinline__ Sym6 body_sym() {
  constexpr rmx::SymC I = rmx::body_i(J);
  Sym6 O;
#pragma unroll
  for (int i = 0; i < 6; ++i) { O.A[i] = I.A[i]; O.C[i] = I.C[i]; }
#pragma unroll
  for (int i = 0; i < 9; ++i) O.B[i] = I.B[i];
  return O;
}
template <int J> __device__ __forceinline__ Sym6 body_plus(const Sym6 &S) {
  constexpr rmx::SymC I = rmx::body_i(J);
  Sym6 O;
  sfor<0, 6>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (I.A[i] == 0.0f) O.A[i] = S.A[i];
    else O.A[i] = I.A[i] + S.A[i];
    if constexpr (I.C[i] == 0.0f) O.C[i] = S.C[i];
    else O.C[i] = I.C[i] + S.C[i];
  });
  sfor<0, 9>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (I.B[i] == 0.0f) O.B[i] = S.B[i];
    else O.B[i] = I.B[i] + S.B[i];
  });
  return O;
}

// body J's centre of mass, and R c_J
template <int J> struct ComC {
  static constexpr float v[3] = {rm::COM[J][0], rm::COM[J][1], rm::COM[J][2]};
};
template <int J> __device__ __forceinline__ V3f rot_com(const M3f &R) {
  return v3(cdot3<ComC<J>>(R.r0), cdot3<ComC<J>>(R.r1), cdot3<ComC<J>>(R.r2));
}

// r_J x w, and Rp r_J (the joint's origin in the parent's world frame)
template <int J> __device__ __forceinline__ V3f rx_c(V3f w) {
  return v3(cdot3<RxRow<J, 0>>(w), cdot3<RxRow<J, 1>>(w), cdot3<RxRow<J, 2>>(w));
}
template <int J> __device__ __forceinline__ V3f rot_org(const M3f &Rp) {
  return v3(cdot3<Org<J>>(Rp.r0), cdot3<Org<J>>(Rp.r1), cdot3<Org<J>>(Rp.r2));
}

// Joint J at q: the generic JT (k, c, s, r), with r the constant origin for a
// revolute joint.
template <int J> __device__ __forceinline__ JT joint_t(float q) {
  JT X;
  X.k = rmx::kax(J);
  constexpr float sg = rmx::sgn(J);
  V3f r = v3(rm::ORIGIN[J][0], rm::ORIGIN[J][1], rm::ORIGIN[J][2]);
  if constexpr (rmx::rev(J)) {
    float sn, cs;
    sincos_rad(q, &sn, &cs);
    X.c = cs;
    X.s = sg * sn;
  } else {
    X.c = 1.0f;
    X.s = 0.0f;
    const float d = sg * q;
    cset<rmx::kax(J)>(r, cget<rmx::kax(J)>(r) + d);
  }
  X.r = r;
  return X;
}

// Joint J with the cosine and sine of a revolute joint given (as the first
// pass stored them), or at q for a prismatic one.
template <int J> __device__ __forceinline__ JT joint_cs(float q, float c, float s) {
  if constexpr (rmx::rev(J)) {
    JT X;
    X.k = rmx::kax(J);
    X.c = c;
    X.s = s;
    X.r = v3(rm::ORIGIN[J][0], rm::ORIGIN[J][1], rm::ORIGIN[J][2]);
    return X;
  } else {
    return joint_t<J>(q);
  }
}

// child -> parent motion transform [E w; E (v - r x w)], E = R^T
template <int J> __device__ __forceinline__ SV x_motion_t(const JT &X, SV m) {
  constexpr int K = rmx::kax(J);
  if constexpr (rmx::rev(J)) return sv(rot_k<K>(X.c, -X.s, m.a), rot_k<K>(X.c, -X.s, m.b - rx_c<J>(m.a)));
  else return x_motion_k<K>(X, m);
}
// X^T f = [R n + r x R f; R f]
template <int J> __device__ __forceinline__ SV x_force_T_t(const JT &X, SV f) {
  constexpr int K = rmx::kax(J);
  if constexpr (rmx::rev(J)) {
    const V3f ff = rot_k<K>(X.c, X.s, f.b);
    return sv(rot_k<K>(X.c, X.s, f.a) + rx_c<J>(ff), ff);
  } else {
    return x_force_T_k<K>(X, f);
  }
}
// S_J x (a motion vector with one nonzero component)
template <int J> __device__ __forceinline__ SV s_vec_t(float x) {
  constexpr int k = rmx::sub_idx(J);
  const float v = rmx::sgn(J) * x;
  return sv(v3(k == 0 ? v : 0.0f, k == 1 ? v : 0.0f, k == 2 ? v : 0.0f),
            v3(k == 3 ? v : 0.0f, k == 4 ? v : 0.0f, k == 5 ? v : 0.0f));
}
template <int J> __device__ __forceinline__ float s_comp_t(SV x) {
  constexpr int k = rmx::sub_idx(J);
  const float c = k == 0 ? x.a.x : k == 1 ? x.a.y : k == 2 ? x.a.z : k == 3 ? x.b.x : k == 4 ? x.b.y : x.b.z;
  return rmx::sgn(J) * c;
}
// v x (S_J x): with S_J = +-e_K in one part, each cross product with e_K has
// two nonzero components
template <int K> __device__ __forceinline__ V3f cross_e(V3f a, float s) {  // a x (s e_K)
  constexpr int I = (K + 1) % 3, Jx = (K + 2) % 3;
  V3f o = v3(0.0f, 0.0f, 0.0f);
  cset<I>(o, cget<Jx>(a) * s);
  cset<Jx>(o, -(cget<I>(a) * s));
  return o;
}
template <int J> __device__ __forceinline__ SV crm_s(SV v, float qd) {
  constexpr int K = rmx::kax(J);
  const float s = rmx::sgn(J) * qd;
  if constexpr (rmx::rev(J)) return sv(cross_e<K>(v.a, s), cross_e<K>(v.b, s));
  else return sv(v3(0.0f, 0.0f, 0.0f), cross_e<K>(v.a, s));
}
// the components of c_J that are not zero by structure: bit i of the mask
// (i = 0..5 over [w; v]); body 2's and the fingers' angular parts vanish
// (their parents do not rotate relative to them, or they slide), and an
// axis-K joint's K components vanish in both parts
template <int J> constexpr unsigned c_mask() {
  constexpr int K = rmx::kax(J);
  unsigned m = 0u;
  for (int i = 0; i < 3; ++i) {
    if (i == K) continue;
    if (rmx::rev(J) && J != 2) m |= 1u << i;
    m |= 1u << (3 + i);
  }
  return J < 2 ? 0u : m;
}
// I c with c's structural zeros (the clear bits of MASK, nonzero) left out
template <unsigned MASK> __device__ __forceinline__ SV sym_mul_masked(const Sym6 &I, SV c) {
  static_assert(MASK != 0u, "an all-zero vector");
  constexpr int first = __builtin_ctz(MASK);
  const float x[6] = {c.a.x, c.a.y, c.a.z, c.b.x, c.b.y, c.b.z};
  float o[6];
  sfor<0, 6>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    float acc = 0.0f;
    sfor<0, 6>([&](auto cc) {
      constexpr int col = decltype(cc)::value;
      if constexpr ((MASK >> col) & 1u) {
        float e;
        if constexpr (r < 3 && col < 3) e = I.A[sidx(r, col)];
        else if constexpr (r < 3) e = I.B[3 * r + (col - 3)];
        else if constexpr (col < 3) e = I.B[3 * col + (r - 3)];
        else e = I.C[sidx(r - 3, col - 3)];
        if constexpr (col == first) acc = e * x[col];
        else acc = fmaf(e, x[col], acc);
      }
    });
    o[r] = acc;
  });
  return sv(v3(o[0], o[1], o[2]), v3(o[3], o[4], o[5]));
}

// I - U U^T / D with U / D formed once: each entry one fused multiply-add
// (the generic form multiplies u_a u_b, then by 1 / D, then subtracts)
__device__ __forceinline__ void sym_rank1_t(Sym6 &I, SV U, float dinv) {
  const float u[6] = {U.a.x, U.a.y, U.a.z, U.b.x, U.b.y, U.b.z};
  float w[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) w[i] = u[i] * dinv;
  const int sx[6] = {0, 0, 0, 1, 1, 2}, sy[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    I.A[i] = fmaf(-w[sx[i]], u[sy[i]], I.A[i]);
    I.C[i] = fmaf(-w[3 + sx[i]], u[3 + sy[i]], I.C[i]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) I.B[3 * r + c] = fmaf(-w[r], u[3 + c], I.B[3 * r + c]);
}

// The translation part of X^T I X for a revolute joint J (constant origin r),
// after the rotation: A'' = A' + rx B'^T - B' rx - rx C' rx, B'' = B' + rx C'.
template <int J> __device__ __forceinline__ Sym6 shift_t(const Sym6 &R) {
  const float *C = R.C;
  const float Cf[9] = {C[0], C[1], C[2], C[1], C[3], C[4], C[2], C[4], C[5]};
  float M[9];  // rx C'
  sfor<0, 3>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
#pragma unroll
    for (int c = 0; c < 3; ++c) M[3 * i + c] = cdot3<RxRow<J, i>>(v3(Cf[c], Cf[3 + c], Cf[6 + c]));
  });
  float N[9], P[9], Q[9];  // rx B'^T, B' rx, M rx
  sfor<0, 3>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
#pragma unroll
    for (int c = 0; c < 3; ++c) N[3 * i + c] = cdot3<RxRow<J, i>>(v3(R.B[3 * c], R.B[3 * c + 1], R.B[3 * c + 2]));
  });
  sfor<0, 3>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      P[3 * i + j] = cdot3<RxCol<J, j>>(v3(R.B[3 * i], R.B[3 * i + 1], R.B[3 * i + 2]));
      Q[3 * i + j] = cdot3<RxCol<J, j>>(v3(M[3 * i], M[3 * i + 1], M[3 * i + 2]));
    }
  });
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
// X^T I X for joint J
template <int J> __device__ __forceinline__ Sym6 congruence_t(const JT &X, const Sym6 &S) {
  constexpr int K = rmx::kax(J);
  if constexpr (!rmx::rev(J)) {
    return congruence_k<K>(X, S);
  } else {
    constexpr int I = (K + 1) % 3, Jx = (K + 2) % 3;
    const float c = X.c, s = X.s, cc = c * c, ss = s * s, cs = c * s;
    Sym6 R;
    rot_sym_k<K>(c, s, cc, ss, cs, S.A, R.A);
    rot_sym_k<K>(c, s, cc, ss, cs, S.C, R.C);
    float P[9];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      P[3 * I + n] = c * S.B[3 * I + n] - s * S.B[3 * Jx + n];
      P[3 * Jx + n] = s * S.B[3 * I + n] + c * S.B[3 * Jx + n];
      P[3 * K + n] = S.B[3 * K + n];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      R.B[3 * m + I] = c * P[3 * m + I] - s * P[3 * m + Jx];
      R.B[3 * m + Jx] = s * P[3 * m + I] + c * P[3 * m + Jx];
      R.B[3 * m + K] = P[3 * m + K];
    }
    return shift_t<J>(R);
  }
}

// World poses of bodies 0..PALM for the arm kinematics (chain_fk with the
// model's constants).
__device__ __forceinline__ void chain_fk_t(const float *q, M3f *Rw, V3f *pw) {
  M3f Rp;
  Rp.r0 = v3(1.0f, 0.0f, 0.0f); Rp.r1 = v3(0.0f, 1.0f, 0.0f); Rp.r2 = v3(0.0f, 0.0f, 1.0f);
  V3f pp = v3(0.0f, 0.0f, 0.0f);
  sfor<0, PALM + 1>([&](auto jc) {
    constexpr int J = decltype(jc)::value;
    const JT X = joint_t<J>(q[J]);
    if constexpr (rmx::rev(J)) pp = pp + rot_org<J>(Rp);
    else pp = pp + mul(Rp, X.r);
    Rp = rot_right_k<rmx::kax(J)>(Rp, X.c, X.s);
    Rw[J] = Rp;
    pw[J] = pp;
  });
}

// Damped least squares on the arm joints 3..8 toward (pt, Rt) (SPEC: the
// kinematics of the robot model):
// dq = J^T (J J^T + lambda^2 I)^-1 e, e = (pt - p_ee, 1/2 sum_k r_k x rt_k).
template <bool SPEC> __device__ __forceinline__ void ik_dls(CScene &sc, float *q, V3f pt, const M3f &Rt) {
  const float lam2 = sc.ik_lambda * sc.ik_lambda;
  for (int it = 0; it < sc.ik_iters; ++it) {
    M3f Rw[PALM + 1];
    V3f pw[PALM + 1];
    if constexpr (SPEC) chain_fk_t(q, Rw, pw);
    else chain_fk(sc, q, Rw, pw);
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
      // the joint's axis in the world (with the model, a signed column of Rw[j])
      const int ax = SPEC ? rm::AXIS[j] : sc.j_axis[j], k = ax % 3;
      const float sg = ax < 3 ? 1.0f : -1.0f;
      const V3f z = SPEC ? sg * col(Rw[j], k)
                         : mul(Rw[j], v3(k == 0 ? sg : 0.0f, k == 1 ? sg : 0.0f, k == 2 ? sg : 0.0f));
      const V3f jv = cross(z, pe - pw[j]);
      J[0][c] = jv.x; J[1][c] = jv.y; J[2][c] = jv.z;
      J[3][c] = z.x; J[4][c] = z.y; J[5][c] = z.z;
    }
    // J J^T + lambda^2 I: its lower triangle (the matrix is symmetric)
    float A[6][6];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c <= r; ++c) {
        float acc = r == c ? lam2 : 0.0f;
#pragma unroll
        for (int k = 0; k < NARM; ++k) acc += J[r][k] * J[c][k];
        A[r][c] = acc;
      }
    // Cholesky solve; each pivot's reciprocal from the hardware's reciprocal
    // square root (about 1 ulp; the matrix is positive definite, d >= lambda^2)
    float L[6][6], inv[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float d = A[j][j];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
      inv[j] = __builtin_amdgcn_rsqf(d);
      L[j][j] = d * inv[j];
#pragma unroll
      for (int i = j + 1; i < 6; ++i) {
        float t = A[i][j];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
        L[i][j] = t * inv[j];
      }
    }
    float y[6], x[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      float t = e[i];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
      y[i] = t * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      float t = y[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) t -= L[k][i] * x[k];
      x[i] = t * inv[i];
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


}  // namespace
}  // namespace cem
